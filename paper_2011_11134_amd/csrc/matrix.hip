// matrix.hip -- IoU matrices (one block a.count x b.count, or ragged segments
// such as per-scene self-pairs of 3D boxes, Sec. IV-A case study at scale) and
// their backward from the saved per-pair state (Sec. II-B: nx and xflags).
//
// The forward is split by register pressure into lean cull kernels and one
// dense exact kernel, with no shared counter anywhere:
//   k_matrix_cull -- one wavefront per tile of R rows x 2048 / R columns of
//     one segment (R = 4, 8 or 16, chosen per call: the autotuner weighs
//     longer contiguous output rows against more column-bound loads per
//     pair).  The rows' axis-aligned bounds (and z-extents)
//     sit in scalar registers; each lane bounds its column boxes 64 at a
//     time, tests them against the rows, writes every pair's initial value
//     (0, or the self diagonal's 1) straight to the output row segments
//     (coalesced), and records the tile's survivor mask and count.
//   k_scan_totals, k_scan_apply -- exclusive prefix of the tile counts in two
//     parallel passes (k_scan_small: in one workgroup, for at most 8192
//     tiles), so the work list is laid out tile by tile, deterministically.
//   k_matrix_fill -- reads the masks; survivors go to their tile's range.
//   k_matrix_exact -- one lane per survivor with every lane busy: the exact
//     pair forward, the IoU written to its place in the output, nx / xflags
//     kept in the work list for the backward.
// A persistent grid walks the tiles of all segments (a prefix sum of tiles per
// segment computed on the device by k_seg_prep, so everything is
// graph-capturable).  The backward (k_matrix_bwd) gives one wavefront a row
// group of 8 rows, whatever the tile shape: the entries of the tile rows
// that cover it are one contiguous range of the work list; each step's row
// gradients are summed without atomics (sorted by row in LDS, each lane
// adding up one (row, vertex) run in a fixed order) and every row is written
// once.  Self pairs need
// nothing else: entries (i, k) and (k, i) are one unordered pair evaluated with
// the lower index first, so the row role of either entry is that pair's
// gradient for the row's box, weighted by both entries' upstream gradients;
// for two different sets the column gradients are added with global atomics.
#include <algorithm>
#include <mutex>
#include <type_traits>
#include <utility>

#include "geom.hpp"
#include "internal.hpp"

namespace dgal {

constexpr int kTilePairs = DGAL_TILE_PAIRS;
constexpr int kGroupRows = 8;     // rows of a backward row group
constexpr int kCullBlock = 256;   // four independent wavefronts
constexpr int kScanBlock = 1024;
constexpr int kExactBlock = 256;
constexpr int kMaxSeg = DGAL_MAX_SEGMENTS;
static_assert(kTilePairs == 2048, "32 words of survivor bits per tile");

// log2 of a supported tile row count (4, 8, 16), or -1.
inline int tile_rows_log2(int rows) {
  return rows == 4 ? 2 : (rows == 8 ? 3 : (rows == 16 ? 4 : -1));
}

struct Segment {
  int64_t a0, b0, na, nb, out0;
  bool ok;
};

struct SegArgs {
  const int64_t* a_off;  // NULL => one segment
  const int64_t* b_off;
  const int64_t* out_off;
  int nseg;
  int64_t a_count, b_count, out_size;
  int self_pairs;
  const int64_t* tile_prefix;   // [nseg+1] (segmented), from k_seg_prep
  const int64_t* group_prefix;  // [nseg+1] row groups (segmented), from k_seg_prep
  int rows_log2;                // tiles of 2^rows_log2 rows x 2^(11 - rows_log2) columns
};

__device__ __forceinline__ Segment load_segment(const SegArgs& a, int s) {
  Segment g;
  if (a.a_off == nullptr) {
    g.a0 = 0;
    g.b0 = 0;
    g.na = a.a_count;
    g.nb = a.b_count;
    g.out0 = 0;
    g.ok = true;
    return g;
  }
  const int64_t a0 = a.a_off[s], a1 = a.a_off[s + 1], b0 = a.b_off[s], b1 = a.b_off[s + 1];
  const int64_t o0 = a.out_off[s];
  g.a0 = a0;
  g.b0 = b0;
  g.na = a1 - a0;
  g.nb = b1 - b0;
  g.out0 = o0;
  g.ok = a0 >= 0 && a1 >= a0 && a1 <= a.a_count && b0 >= 0 && b1 >= b0 && b1 <= a.b_count &&
         o0 >= 0 && o0 <= a.out_size && g.nb < (1 << 24) &&
         (g.nb == 0 || g.na <= (a.out_size - o0) / g.nb) &&
         (!a.self_pairs || (a0 == b0 && a1 == b1));
  if (s > 0) {  // blocks are laid out in segment order without overlap
    const int64_t pna = a.a_off[s] - a.a_off[s - 1], pnb = a.b_off[s] - a.b_off[s - 1];
    g.ok = g.ok && o0 >= a.out_off[s - 1] + pna * pnb;
  }
  return g;
}

// Backward row groups, tile rows and tile columns of a segment.
__device__ __forceinline__ int64_t groups_of(const Segment& g) {
  return (g.na > 0 && g.nb > 0) ? (g.na + kGroupRows - 1) / kGroupRows : 0;
}
__device__ __forceinline__ int64_t tile_rows_of(const Segment& g, int rl) {
  return (g.na > 0 && g.nb > 0) ? (g.na + (1 << rl) - 1) >> rl : 0;
}
__device__ __forceinline__ int64_t col_tiles_of(const Segment& g, int rl) {
  const int cl = 11 - rl;
  return (g.nb + (1 << cl) - 1) >> cl;
}

// Tile and row-group prefixes over segments (one workgroup).  Rejected
// segments own nothing and raise kErrSegment.
__global__ __launch_bounds__(256) void k_seg_prep(SegArgs a, int* err, int64_t* tile_prefix,
                                                  int64_t* group_prefix) {
  __shared__ int64_t part_t[256], part_g[256];
  const int tid = threadIdx.x;
  const int per = (a.nseg + 255) / 256;
  const int s0 = min(a.nseg, tid * per), s1 = min(a.nseg, s0 + per);
  int64_t st = 0, sg = 0;
  for (int s = s0; s < s1; ++s) {
    const Segment g = load_segment(a, s);
    if (!g.ok) {
      atomicOr(err, kErrSegment);
      continue;
    }
    sg += groups_of(g);
    st += tile_rows_of(g, a.rows_log2) * col_tiles_of(g, a.rows_log2);
  }
  part_t[tid] = st;
  part_g[tid] = sg;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {  // inclusive scans
    const int64_t vt = tid >= d ? part_t[tid - d] : 0;
    const int64_t vg = tid >= d ? part_g[tid - d] : 0;
    __syncthreads();
    part_t[tid] += vt;
    part_g[tid] += vg;
    __syncthreads();
  }
  int64_t rt = tid > 0 ? part_t[tid - 1] : 0, rg = tid > 0 ? part_g[tid - 1] : 0;
  if (tid == 0) {
    tile_prefix[0] = 0;
    group_prefix[0] = 0;
  }
  for (int s = s0; s < s1; ++s) {
    const Segment g = load_segment(a, s);
    if (g.ok) {
      rg += groups_of(g);
      rt += tile_rows_of(g, a.rows_log2) * col_tiles_of(g, a.rows_log2);
    }
    tile_prefix[s + 1] = rt;
    group_prefix[s + 1] = rg;
  }
}

// Last s with prefix[s] <= v (the segment that owns item v of a prefix).
__device__ __forceinline__ int find_segment(const int64_t* prefix, int nseg, int64_t v) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The same search by a whole wavefront, for a wave-uniform v: each round
// loads up to 64 evenly spaced entries of the remaining range (one a lane)
// and keeps the span from the last one not past v, so up to 64 segments take
// one round of loads and up to 4096 two (the scalar search above takes a
// dependent load per halving).
__device__ __forceinline__ int wave_find_segment(const int64_t* prefix, int nseg, int64_t v) {
  const int lane = threadIdx.x & 63;
  int lo = 0, hi = nseg;  // the answer lies in [lo, hi)
  while (hi - lo > 1) {
    const int step = (hi - lo + 63) >> 6;
    const int i = lo + lane * step;
    const uint64_t m = __ballot(i < hi && prefix[i] <= v);
    const int k = m != 0ull ? 63 - __clzll(m) : 0;
    lo += k * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

// Axis-aligned bounds and z-extent of one box (padded slots repeat vertex 0,
// so the bounds over all K slots are the polygon's).
struct Bounds {
  float x0, y0, x1, y1, lo, hi;
};

template <int K, bool FIXED, bool Z3>
__device__ __forceinline__ Bounds box_bounds(const PolyArgs& p, int64_t idx) {
  Poly<K> P;
  const int n = FIXED ? K : poly_count(p.nv, idx, p.kmax);
  load_poly<K, FIXED>(p.xy, idx, p.kmax, p.vec4, n, P);
  Bounds b;
  b.x0 = b.x1 = P.x[0];
  b.y0 = b.y1 = P.y[0];
#pragma unroll
  for (int k = 1; k < K; ++k) {
    b.x0 = fminf(b.x0, P.x[k]);
    b.x1 = fmaxf(b.x1, P.x[k]);
    b.y0 = fminf(b.y0, P.y[k]);
    b.y1 = fmaxf(b.y1, P.y[k]);
  }
  b.lo = Z3 ? p.zlo[idx] : 0.f;
  b.hi = Z3 ? p.zhi[idx] : 0.f;
  return b;
}

__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct CullArgs {
  SegArgs seg;
  PolyArgs a, b;
  int64_t single_tiles;
  float* iou;
  int64_t* pair_id;
  int64_t capacity;
  int64_t* tile_start;
  int32_t* tile_count;
  int64_t tile_capacity;
  uint64_t* tile_mask;  // [tile_capacity][kMaskWords]
  int* err;
};

constexpr int kBitWords = kTilePairs / 64;  // survivor bits of a tile
constexpr int kMaskWords = DGAL_TILE_MASK_WORDS;            // + tile origin + row length
static_assert(kMaskWords == kBitWords + 2 && kMaskWords <= 64, "mask words");

// Segment s without the checks of load_segment: the tile walk only reaches
// segments that k_seg_prep accepted.
__device__ __forceinline__ Segment tile_segment(const SegArgs& a, int s) {
  Segment g;
  if (a.a_off == nullptr) {
    g.a0 = 0;
    g.b0 = 0;
    g.na = a.a_count;
    g.nb = a.b_count;
    g.out0 = 0;
  } else {
    g.a0 = a.a_off[s];
    g.b0 = a.b_off[s];
    g.na = a.a_off[s + 1] - g.a0;
    g.nb = a.b_off[s + 1] - g.b0;
    g.out0 = a.out_off[s];
  }
  g.ok = true;
  return g;
}

// Sign bit of the difference hi - lo: set when lo > hi, clear when they are
// equal (the closed test keeps touching boxes).
__device__ __forceinline__ uint32_t gap_bits(float hi, float lo) {
  return __float_as_uint(hi - lo);
}

template <int N, class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>()), ...);
}
// f(0), f(1), ..., f(N - 1) with compile-time arguments.
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl<N>(f, std::make_integer_sequence<int, N>());
}

// v_writelane: `val` (wave-uniform) into lane L (a constant) of `old`.
template <int L>
__device__ __forceinline__ uint32_t write_lane(uint32_t old, uint32_t val) {
  static_assert(L >= 0 && L < 64, "lane");
  asm("v_writelane_b32 %0, %1, %2" : "+v"(old) : "s"(val), "n"(L));
  return old;
}

// The largest float below v (finite v): lo < v <=> lo <= below(v), so the
// open z test becomes the closed one on a lowered upper end.
__device__ __forceinline__ float below(float v) {
  const uint32_t b = __float_as_uint(v);
  if ((b & 0x7fffffffu) == 0u) return -1.40129846e-45f;  // +-0 -> -denorm_min
  return __uint_as_float((int32_t)b > 0 ? b - 1u : b + 1u);
}

// Walks a contiguous range of tiles: the segment is searched once, then
// followed tile by tile (row-major within a segment, segments in order), so
// that a tile costs no search and no division.
template <int R>
struct TileCursor {
  static constexpr int C = kTilePairs / R;
  static constexpr int RL = R == 4 ? 2 : (R == 8 ? 3 : 4);
  int s;
  int64_t seg_end;  // first tile past segment s
  Segment g;
  int64_t nct, tr, tc;

  __device__ void load(const SegArgs& seg, bool segmented) {
    g = tile_segment(seg, s);
    nct = col_tiles_of(g, RL);
    seg_end = segmented ? seg.tile_prefix[s + 1] : (int64_t)0x7fffffffffffffff;
  }
  __device__ void seek(const SegArgs& seg, bool segmented, int64_t u) {
    s = segmented ? wave_find_segment(seg.tile_prefix, seg.nseg, u) : 0;
    load(seg, segmented);
    const int64_t lu = segmented ? u - seg.tile_prefix[s] : u;
    tr = lu / nct;
    tc = lu - tr * nct;
  }
  // to tile u + 1 (u the current tile)
  __device__ void next(const SegArgs& seg, bool segmented, int64_t u) {
    if (++tc == nct) {
      tc = 0;
      ++tr;
    }
    if (u + 1 >= seg_end) {  // the next non-empty segment
      do {
        ++s;
      } while (s < seg.nseg && seg.tile_prefix[s + 1] <= u + 1);
      if (s < seg.nseg) {
        load(seg, segmented);
        tr = 0;
        tc = 0;
      }
    }
  }
  __device__ int64_t r0() const { return tr * R; }
  __device__ int64_t cb() const { return tc * C; }
};

// The contiguous range of tiles of wavefront `wid` out of `nw`.
__device__ __forceinline__ void wave_tiles(int64_t total, int64_t wid, int64_t nw, int64_t& u0,
                                           int64_t& u1) {
  const int64_t per = (total + nw - 1) / nw;
  u0 = wid * per;
  u1 = u0 + per < total ? u0 + per : total;
}

// Count pass: writes every pair of the tile (0 for the culled ones, which
// stays, or 1 on the self diagonal; the exact kernel later overwrites the
// survivors), the tile's survivor mask (kMaskWords words, chunk-major) and its
// survivor count.  The tile walk is wave-uniform, so its indices, the segment
// and the rows' bounds live in scalar registers.  The test of a (row, column)
// pair is one OR of the sign bits of its four (2D) or six (3D) bound
// differences, so that the vector unit does the work and the scalar unit only
// counts: overlapping closed boxes (touching ones go to the exact kernel)
// with overlapping open z extents (a closed test against upper ends lowered
// by one ulp) survive; invalid columns and rows, and empty z extents, carry
// x1 = -inf.
template <int K, bool FIXED, bool Z3, int R>
__global__ __launch_bounds__(kCullBlock) void k_matrix_cull(CullArgs m) {
  constexpr int WAVES = kCullBlock / 64;
  constexpr int C = kTilePairs / R;
  static_assert(R == 4 || R == 8 || R == 16, "tile rows");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool segmented = m.seg.a_off != nullptr;
  const int64_t total = segmented ? m.seg.tile_prefix[m.seg.nseg] : m.single_tiles;

  int64_t u0, u1;
  wave_tiles(total, (int64_t)blockIdx.x * WAVES + wave, (int64_t)gridDim.x * WAVES, u0, u1);
  TileCursor<R> cur;
  if (u0 < u1) cur.seek(m.seg, segmented, u0);
  // the rows' bounds, in scalar registers, kept while the tiles of a range
  // stay in one tile row (the usual case: a range is a few tiles)
  Bounds rb[R];
  int64_t rows_of = -1;  // first row (in a) whose bounds rb holds
  for (int64_t u = u0; u < u1; cur.next(m.seg, segmented, u), ++u) {
    const Segment& g = cur.g;
    const int64_t r0 = cur.r0(), cb = cur.cb();
    const int nr = (int)min((int64_t)R, g.na - r0);
    const int64_t ce = min(g.nb, cb + C);
    float* out_rows = m.iou + g.out0 + r0 * g.nb;

    if (g.a0 + r0 != rows_of) {  // uniform
      // row bounds: lane j < nr bounds row j, then every lane holds all of them
      rows_of = g.a0 + r0;
      Bounds rl = {0.f, 0.f, -1.f, -1.f, 0.f, 0.f};
      if (lane < nr) rl = box_bounds<K, FIXED, Z3>(m.a, g.a0 + r0 + lane);
      if (lane >= nr || (Z3 && !(rl.hi > rl.lo))) rl.x1 = -__builtin_inff();
      if (Z3) rl.hi = below(rl.hi);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        rb[j].x0 = lane_bcast(rl.x0, j);
        rb[j].y0 = lane_bcast(rl.y0, j);
        rb[j].x1 = lane_bcast(rl.x1, j);
        rb[j].y1 = lane_bcast(rl.y1, j);
        rb[j].lo = lane_bcast(rl.lo, j);
        rb[j].hi = lane_bcast(rl.hi, j);
      }
    }
    uint32_t n = 0;         // survivors so far (uniform; at most kTilePairs)
    uint32_t mlo = 0u, mhi = 0u;  // lane w < kBitWords: mask word w of the tile
    // the next 64 column boxes are loaded while the current ones are tested
    Bounds nxt = {0.f, 0.f, -1.f, -1.f, 0.f, 0.f};
    if (cb + lane < ce) nxt = box_bounds<K, FIXED, Z3>(m.b, g.b0 + cb + lane);
    static_for<C / 64>([&](auto cic) {
      constexpr int ci = decltype(cic)::value;
      const int64_t c0 = cb + ci * 64;
      if (c0 >= ce) return;  // uniform; so are the later chunks
      const bool valid = c0 + lane < ce;
      Bounds cbx = nxt;
      if (c0 + 64 + lane < ce) nxt = box_bounds<K, FIXED, Z3>(m.b, g.b0 + c0 + 64 + lane);
      if (!valid || (Z3 && !(cbx.hi > cbx.lo))) cbx.x1 = -__builtin_inff();
      if (Z3) cbx.hi = below(cbx.hi);
      // the self diagonal crosses this chunk at lane r0 + j - c0
      const int64_t dd = r0 - c0;
      const bool dchunk = m.seg.self_pairs && dd > -R && dd < 64;
      uint64_t mk[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        uint32_t bits = gap_bits(rb[j].x1, cbx.x0) | gap_bits(cbx.x1, rb[j].x0) |
                        gap_bits(rb[j].y1, cbx.y0) | gap_bits(cbx.y1, rb[j].y0);
        if (Z3) bits |= gap_bits(rb[j].hi, cbx.lo) | gap_bits(cbx.hi, rb[j].lo);
        // rows and columns past the block never survive, whatever the
        // infinities of the other side's bounds make of the test
        mk[j] = j < nr ? __ballot(valid && (int32_t)bits >= 0) : 0ull;
      }
      if (dchunk) {  // rare: the chunk holds part of the diagonal
        const int d = (int)dd;
#pragma unroll
        for (int j = 0; j < R; ++j)
          if (d + j >= 0 && d + j < 64) mk[j] &= ~(1ull << (d + j));
      }
      // word ci * R + j of the tile goes to that lane
      static_for<R>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        mlo = write_lane<ci * R + j>(mlo, (uint32_t)mk[j]);
        mhi = write_lane<ci * R + j>(mhi, (uint32_t)(mk[j] >> 32));
        n += (uint32_t)__popcll(mk[j]);
      });
    });
    // the tile's output rows, each one contiguous run of up to 256 values (0,
    // or 1 where a self block's diagonal crosses); the exact kernel later
    // overwrites the survivors
    const int64_t dg = m.seg.self_pairs ? r0 - cb : INT64_MIN / 2;  // diagonal column of row 0
    for (int j = 0; j < nr; ++j) {
      float* row = out_rows + (int64_t)j * g.nb + cb;
      const bool drow = dg + j >= 0 && dg + j < C;  // uniform
#pragma unroll
      for (int ci = 0; ci < C / 64; ++ci) {
        const int col = ci * 64 + lane;
        if (cb + col < ce) row[col] = (drow && col == dg + j) ? 1.f : 0.f;
      }
    }
    if (u < m.tile_capacity) {
      // the tile's state for the fill pass: bits, origin, row length
      uint64_t mword = ((uint64_t)mhi << 32) | mlo;
      if (lane == kBitWords) mword = (uint64_t)(g.out0 + r0 * g.nb + cb);
      if (lane == kBitWords + 1) mword = (uint64_t)g.nb;
      if (lane < kMaskWords) m.tile_mask[u * kMaskWords + lane] = mword;
      if (lane == 0) m.tile_count[u] = (int32_t)n;
    } else if (lane == 0) {
      atomicOr(m.err, kErrCapacity);
    }
  }
}

// Fill pass: the survivors' output indices, read from the tile state the
// count pass wrote (bits, origin, row length), go to the tile's range of the
// work list (chunk-major, the order of the bits): lane w writes the bits of
// word w, from the exclusive prefix of the words' counts.  A tile costs one
// round of independent loads (prefetched), no segment lookup.
__global__ __launch_bounds__(kCullBlock) void k_matrix_fill(CullArgs m) {
  constexpr int WAVES = kCullBlock / 64;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool segmented = m.seg.a_off != nullptr;
  int64_t total = segmented ? m.seg.tile_prefix[m.seg.nseg] : m.single_tiles;
  total = total < m.tile_capacity ? total : m.tile_capacity;
  int64_t u0, u1;
  wave_tiles(total, (int64_t)blockIdx.x * WAVES + wave, (int64_t)gridDim.x * WAVES, u0, u1);
  // the next tile's state and start are loaded while this tile is written
  uint64_t word_next = 0ull;
  int64_t start_next = 0;
  if (u0 < u1) {
    word_next = lane < kMaskWords ? m.tile_mask[u0 * kMaskWords + lane] : 0ull;
    start_next = m.tile_start[u0];
  }
  for (int64_t u = u0; u < u1; ++u) {
    const uint64_t word = word_next;
    const int64_t start = start_next;
    if (u + 1 < u1) {
      word_next = lane < kMaskWords ? m.tile_mask[(u + 1) * kMaskWords + lane] : 0ull;
      start_next = m.tile_start[u + 1];
    }
    const uint64_t bits = lane < kBitWords ? word : 0ull;
    if (__ballot(bits != 0ull) == 0ull) continue;  // uniform: an empty tile
    // (the lane reads return int: each half is taken as unsigned, or a low
    // half with its top bit set would sign-extend over the high half)
    const int64_t origin = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(word >> 32), kBitWords) << 32) |
                                     (uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)word, kBitWords));
    const int64_t nb = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(word >> 32), kBitWords + 1) << 32) |
                                 (uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)word, kBitWords + 1));
    // every lane writes the survivors of its own word: its first slot is the
    // exclusive prefix of the words' bit counts
    const int cnt = __popcll(bits);
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < kBitWords; d <<= 1) {
      const int o = __shfl_up(incl, d);
      if (lane >= d) incl += o;
    }
    int64_t slot = start + (incl - cnt);
    const int rl = m.seg.rows_log2;
    const int j = lane & ((1 << rl) - 1), c = lane >> rl;
    const int64_t first = origin + (int64_t)j * nb + c * 64;
    uint64_t w = bits;
    while (w != 0ull) {
      const int b = __builtin_ctzll(w);
      w &= w - 1ull;
      if (slot < m.capacity) m.pair_id[slot] = first + b;
      ++slot;
    }
  }
}

// Exclusive prefix of the tile counts in two parallel passes over chunks of
// kScanChunk tiles: k_scan_totals sums every chunk; k_scan_apply rescans its
// chunk in LDS, adds the totals of the chunks before it, writes tile_start,
// clamps the counts to what the capacity holds and (last chunk) the total.
constexpr int kScanChunk = kScanBlock * 4;

__device__ __forceinline__ int64_t scan_tiles(const int64_t* tile_prefix, int nseg,
                                              int64_t single_tiles, int64_t tile_capacity) {
  const int64_t nt = tile_prefix != nullptr ? tile_prefix[nseg] : single_tiles;
  return nt < tile_capacity ? nt : tile_capacity;
}

// Block-wide inclusive scan of one value per thread (wave scans + LDS).
__device__ __forceinline__ int64_t block_inclusive_scan(int64_t v, int64_t* s_w) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t o = __shfl_up(v, d);
    if (lane >= d) v += o;
  }
  if (lane == 63) s_w[wave] = v;
  __syncthreads();
  int64_t add = 0;
  for (int w = 0; w < wave; ++w) add += s_w[w];
  __syncthreads();
  return v + add;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_totals(const int64_t* tile_prefix, int nseg,
                                                            int64_t single_tiles,
                                                            int64_t tile_capacity,
                                                            const int32_t* tile_count,
                                                            int64_t* totals) {
  __shared__ int64_t s_w[kScanBlock / 64];
  const int64_t nt = scan_tiles(tile_prefix, nseg, single_tiles, tile_capacity);
  const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
  if (c0 >= nt) return;  // uniform
  int64_t v = 0;
#pragma unroll
  for (int k = 0; k < kScanChunk / kScanBlock; ++k) {
    const int64_t t = c0 + k * kScanBlock + threadIdx.x;
    if (t < nt) v += tile_count[t];
  }
  v = block_inclusive_scan(v, s_w);
  if (threadIdx.x == kScanBlock - 1) totals[blockIdx.x] = v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const int64_t* tile_prefix, int nseg,
                                                           int64_t single_tiles,
                                                           int64_t tile_capacity,
                                                           const int64_t* totals,
                                                           int64_t* tile_start,
                                                           int32_t* tile_count, int64_t* count,
                                                           int64_t capacity, int* err) {
  __shared__ int64_t s_w[kScanBlock / 64];
  const int64_t nt = scan_tiles(tile_prefix, nseg, single_tiles, tile_capacity);
  const int64_t nchunks = (nt + kScanChunk - 1) / kScanChunk;
  const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
  if (c0 >= nt) {  // uniform; an empty matrix still publishes its total
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0;
    return;
  }
  // base: totals of the chunks before this one
  int64_t b = 0;
  for (int64_t k = threadIdx.x; k < blockIdx.x; k += kScanBlock) b += totals[k];
  b = block_inclusive_scan(b, s_w);
  __shared__ int64_t s_base;
  if (threadIdx.x == kScanBlock - 1) s_base = b;
  __syncthreads();
  int64_t run = s_base;
  // this chunk: kScanChunk / kScanBlock consecutive tiles per thread
  constexpr int PER = kScanChunk / kScanBlock;
  int64_t c[PER];
  int64_t v = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t t = c0 + (int64_t)threadIdx.x * PER + k;
    c[k] = t < nt ? tile_count[t] : 0;
    v += c[k];
  }
  const int64_t incl = block_inclusive_scan(v, s_w);
  run += incl - v;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t t = c0 + (int64_t)threadIdx.x * PER + k;
    if (t < nt) {
      tile_start[t] = run;
      int64_t room = capacity - run;
      room = room < 0 ? 0 : (room > c[k] ? c[k] : room);
      tile_count[t] = (int32_t)room;
    }
    run += c[k];
  }
  if (blockIdx.x == nchunks - 1 && threadIdx.x == kScanBlock - 1) {
    *count = run;
    if (run > capacity) atomicOr(err, kErrCapacity);
  }
}

// The same exclusive prefix in one workgroup, for tile tables of at most
// kScanSmall entries (a call's tile capacity bounds its tile count): one
// coalesced round of loads into LDS (a tile holds at most 2048 survivors, so
// its count fits 16 bits and a prefix over 8192 tiles 32 bits), the scan of
// each thread's run of 8 tiles, and one coalesced round of stores: one
// launch in place of the two passes.
constexpr int64_t kScanSmall = 8 * kScanBlock;

__global__ __launch_bounds__(kScanBlock) void k_scan_small(const int64_t* tile_prefix, int nseg,
                                                           int64_t single_tiles,
                                                           int64_t tile_capacity,
                                                           int64_t* tile_start,
                                                           int32_t* tile_count, int64_t* count,
                                                           int64_t capacity, int* err) {
  constexpr int PER = kScanSmall / kScanBlock;
  __shared__ uint16_t s_cnt[kScanSmall];
  __shared__ int32_t s_pre[kScanSmall];
  __shared__ int64_t s_w[kScanBlock / 64];
  const int t = threadIdx.x;
  const int64_t nt = scan_tiles(tile_prefix, nseg, single_tiles, tile_capacity);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = k * kScanBlock + t;
    s_cnt[i] = i < nt ? (uint16_t)tile_count[i] : (uint16_t)0;
  }
  __syncthreads();
  int64_t v = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) v += s_cnt[t * PER + k];
  const int64_t incl = block_inclusive_scan(v, s_w);
  int32_t run = (int32_t)(incl - v);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    s_pre[t * PER + k] = run;
    run += s_cnt[t * PER + k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = k * kScanBlock + t;
    if (i < nt) {
      const int64_t start = s_pre[i], c = s_cnt[i];
      tile_start[i] = start;
      int64_t room = capacity - start;
      room = room < 0 ? 0 : (room > c ? c : room);
      tile_count[i] = (int32_t)room;
    }
  }
  if (t == kScanBlock - 1) {
    *count = incl;
    if (incl > capacity) atomicOr(err, kErrCapacity);
  }
}

struct ExactArgs {
  SegArgs seg;
  PolyArgs a, b;
  float* iou;
  const int64_t* pair_id;
  uint8_t* s_nx;
  uint8_t* s_flags;
  int64_t capacity;
  const int64_t* count;
  int cap;
  int* err;
  unsigned long long* stats;  // path statistics (NULL: off)
};

__device__ __forceinline__ int64_t wave_first(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Quotient and remainder of a non-negative index by a positive divisor below
// 2^24 (32-bit division when the index allows it).
__device__ __forceinline__ void divmod(int64_t v, int64_t d, int64_t& q, int64_t& r) {
  if (v < (int64_t)0xffffffff) {
    const uint32_t q32 = (uint32_t)v / (uint32_t)d;
    q = q32;
  } else {
    q = v / d;
  }
  r = v - q * d;
}

// Segment, row and column (within the segment) of a flat output index.  The
// work list is in output order, so the entries of one wavefront mostly share
// a segment: it is searched once for the wavefront's first entry, and a lane
// outside that segment searches for itself.
// The segment a wavefront last located, and its block of the output
// [lo, hi) (empty until the first search; wave-uniform).
struct SegCache {
  Segment g;
  int64_t lo = 0, hi = 0;
};

__device__ __forceinline__ bool locate(const SegArgs& sa, int64_t pid, SegCache& sc, Segment& g,
                                       int64_t& r, int64_t& c) {
  if (sa.a_off == nullptr) {
    g = load_segment(sa, 0);
  } else {
    const int64_t pid0 = wave_first(pid);
    if (!(pid0 >= sc.lo && pid0 < sc.hi)) {  // uniform: a wavefront's entries mostly stay in one
      sc.g = load_segment(sa, wave_find_segment(sa.out_off, sa.nseg, pid0));
      sc.lo = sc.g.out0;
      sc.hi = sc.g.ok ? sc.g.out0 + sc.g.na * sc.g.nb : sc.g.out0;
    }
    g = (pid >= sc.lo && pid < sc.hi) ? sc.g : load_segment(sa, find_segment(sa.out_off, sa.nseg, pid));
  }
  const int64_t local = pid - g.out0;
  if (!g.ok || g.nb <= 0 || local < 0) return false;
  divmod(local, g.nb, r, c);
  return r < g.na;
}

template <int K, bool FIXED, bool Z3>
__global__ __launch_bounds__(kExactBlock)
__attribute__((amdgpu_waves_per_eu(4))) void k_matrix_exact(ExactArgs m) {
  constexpr int CAP = 2 * K;
  __shared__ float2 s_pt[CAP * kExactBlock];
  __shared__ uint16_t s_cd[CAP * kExactBlock];
  const int tid = threadIdx.x;
  int64_t n = *m.count;
  n = n < m.capacity ? n : m.capacity;
  // each wavefront a contiguous range of entries, 64 at a time: consecutive
  // entries mostly share a segment, which is then searched once
  const int64_t wid = ((int64_t)blockIdx.x * kExactBlock + tid) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kExactBlock) >> 6;
  const int64_t per = (((n + nw - 1) / nw) + 63) & ~(int64_t)63;
  const int64_t e_end = min(n, wid * per + per);
  SegCache sc;
  // 4-slot pairs: the next step's ids are loaded while this step's pairs are
  // evaluated (the 8-slot kernel has no registers to spare for them)
  constexpr bool PREFETCH = K == 4;
  int64_t pid_next = 0;
  if (PREFETCH && wid * per + (tid & 63) < e_end) pid_next = m.pair_id[wid * per + (tid & 63)];
  for (int64_t e = wid * per + (tid & 63); e < e_end; e += 64) {
    const int64_t pid = PREFETCH ? pid_next : m.pair_id[e];
    if (PREFETCH && e + 64 < e_end) pid_next = m.pair_id[e + 64];
    Segment g;
    int64_t r = 0, c = 0;
    if (!locate(m.seg, pid, sc, g, r, c)) continue;  // not written by the cull on these shapes
    int64_t ia = g.a0 + r, ib = g.b0 + c;
    if (m.seg.self_pairs && r > c) {  // one unordered pair: the lower index is P
      const int64_t t = ia;
      ia = ib;
      ib = t;
    }
    const int n1 = FIXED ? K : poly_count(m.a.nv, ia, m.a.kmax);
    const int n2 = FIXED ? K : poly_count(m.b.nv, ib, m.b.kmax);
    Poly<K> P, Q;
    load_poly<K, FIXED>(m.a.xy, ia, m.a.kmax, m.a.vec4, n1, P);
    load_poly<K, FIXED>(m.b.xy, ib, m.b.kmax, m.b.vec4, n2, Q);
    PairResult<K> res;
    pair_forward<K, FIXED, kExactBlock>(P, n1, Q, n2, s_pt + tid, s_cd + tid, res);
    count_path(m.stats, res.exact, res.thin);
    m.iou[pid] = pair_iou<Z3>(res.inter, res.a1, res.a2, res.m, m.a.zlo, m.a.zhi, ia, m.b.zlo,
                              m.b.zhi, ib);
    if (res.overflow) atomicOr(m.err, kErrCapacity);
    m.s_nx[e] = (uint8_t)res.m;
    uint8_t* row = m.s_flags + e * (int64_t)m.cap;
#pragma unroll
    for (int b = 0; b < CAP; ++b)
      if (b < m.cap) row[b] = (uint8_t)(res.codes[b >> 2] >> ((b & 3) * 8));
    // rare: the areas again in fp64, from the polygons reloaded, and the IoU
    // written again
    if (res.thin) {
      load_poly<K, FIXED>(m.a.xy, opaque(ia), m.a.kmax, m.a.vec4, n1, P);
      load_poly<K, FIXED>(m.b.xy, opaque(ib), m.b.kmax, m.b.vec4, n2, Q);
      stage_pair<K, kExactBlock>(s_pt + tid, P, Q);
      float inter, a1, a2;
      thin_areas64<K, FIXED, kExactBlock>(res.m, res.codes, n1, n2, s_pt + tid, inter, a1, a2);
      m.iou[pid] = pair_iou<Z3>(inter, a1, a2, res.m, m.a.zlo, m.a.zhi, ia, m.b.zlo, m.b.zhi, ib);
    }
  }
}

// Zero-fills n floats.
__global__ void k_fill_zero(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

struct BwdArgs {
  SegArgs seg;
  PolyArgs a, b;
  int64_t single_groups;
  const float* grad;
  const int64_t* pair_id;
  const uint8_t* s_nx;
  const uint8_t* s_flags;
  int64_t capacity;
  const int64_t* tile_start;
  const int32_t* tile_count;
  int64_t tile_capacity;
  int cap;
  bool flags_vec;  // cap == 2K and s_flags aligned to cap bytes: whole-row loads
  float* ga_xy;
  float* gb_xy;  // unused when self_pairs
  float* ga_z;
  float* gb_z;
};

template <int K>
constexpr int bwd_block() {
  return K == 8 ? 128 : 256;
}

// Sums one step's row gradients (64 entries, each one row's H value pairs:
// a vertex's x and y, or the z-extent's two ends) per (row, pair) into the
// lanes' accumulators without atomics (LDS float atomic adds measured slow
// here: 10 a lane per step cost the c5 backward ~15 us).  The lanes' pairs go
// to the wavefront's own LDS columns ordered by row (the row's offset, then
// the lane's rank among that row's lanes); lane c then adds up the run of
// combination c = (row c / H, pair c % H), and c + 64, ..., in lane order: a
// fixed order, so the sums are the same from run to run.  rl < 0: the lane
// holds nothing.  Called by all 64 lanes.
template <int H, int BLOCK>
__device__ __forceinline__ void step_row_sums(int rl, const float2 (&gv)[H], float2* stage,
                                              float2 (&acc)[(kGroupRows * H + 63) / 64]) {
  constexpr int NACC = (kGroupRows * H + 63) / 64;
  const int lane = threadIdx.x & 63;
  int pos = 0, base = 0, most = 0;
  int off[kGroupRows], cnt[kGroupRows];
#pragma unroll
  for (int r = 0; r < kGroupRows; ++r) {
    const uint64_t mr = __ballot(rl == r);
    const int c = __popcll(mr);
    if (rl == r)
      pos = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mr >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)mr, 0u));
    off[r] = base;
    cnt[r] = c;
    base += c;
    most = max(most, c);
  }
  if (base == 0) return;  // uniform: nothing in this step
  if (rl >= 0) {
#pragma unroll
    for (int h = 0; h < H; ++h) stage[h * BLOCK + pos] = gv[h];
  }
  wave_sync();
#pragma unroll
  for (int j = 0; j < NACC; ++j) {
    const int c = lane + 64 * j;
    const int r = c / H, h = c - r * H;
    int o = 0, n = 0;  // the run of row r (none past the last row)
#pragma unroll
    for (int rr = 0; rr < kGroupRows; ++rr) {
      if (r == rr) {
        o = off[rr];
        n = cnt[rr];
      }
    }
    const float2* run = stage + h * BLOCK + o;
    float sx = 0.f, sy = 0.f;
    for (int i = 0; i < most; ++i) {
      if (i < n) {
        const float2 v = run[i];
        sx += v.x;
        sy += v.y;
      }
    }
    acc[j].x += sx;
    acc[j].y += sy;
  }
  wave_sync();  // the columns are the pair kernels' staging again
}

template <int K, bool FIXED, bool Z3>
__global__ __launch_bounds__(bwd_block<K>())
__attribute__((amdgpu_waves_per_eu(K == 4 ? 4 : 2))) void k_matrix_bwd(BwdArgs m) {
  constexpr int BLOCK = bwd_block<K>();
  constexpr int WAVES = BLOCK / 64;
  constexpr int CAP = 2 * K;
  constexpr int H = K + (Z3 ? 1 : 0);  // a row's value pairs: vertices, then (zlo, zhi)
  constexpr int NACC = (kGroupRows * H + 63) / 64;
  static_assert(H <= CAP, "a step's row values fit the staging columns");
  __shared__ float2 s_v[CAP * BLOCK];
  __shared__ float2 s_g[CAP * BLOCK];
  __shared__ uint2 s_tab[256];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: the row-group walk is scalar
  float2* stage = s_v + wave * 64;  // this wavefront's columns of the staging
  fill_code_table<K, FIXED, BLOCK>(s_tab);
  __syncthreads();
  const bool segmented = m.seg.a_off != nullptr;
  const int64_t total = segmented ? m.seg.group_prefix[m.seg.nseg] : m.single_groups;
  const int kx = m.a.kmax;
  if (segmented) {
    // rows that no row group writes are zeroed here: rows outside every
    // segment, and the rows of a segment without row groups (rejected, or
    // without columns); every other row is written once by its row group
    const int64_t rowlen = (int64_t)kx * 2;
    auto zero_rows = [&](int64_t r0, int64_t r1, int64_t t, int64_t nt) {
      r0 = max(r0, (int64_t)0);
      r1 = min(r1, m.a.count);
      for (int64_t i = r0 * rowlen + t; i < r1 * rowlen; i += nt) m.ga_xy[i] = 0.f;
      if (Z3)
        for (int64_t i = r0 * 2 + t; i < r1 * 2; i += nt) m.ga_z[i] = 0.f;
    };
    const int64_t gt = (int64_t)blockIdx.x * BLOCK + tid, gn = (int64_t)gridDim.x * BLOCK;
    zero_rows(0, m.seg.a_off[0], gt, gn);
    zero_rows(m.seg.a_off[m.seg.nseg], m.a.count, gt, gn);
    for (int s = blockIdx.x; s < m.seg.nseg; s += gridDim.x)
      if (m.seg.group_prefix[s + 1] == m.seg.group_prefix[s])
        zero_rows(m.seg.a_off[s], m.seg.a_off[s + 1], tid, BLOCK);
  }

  for (int64_t u = (int64_t)blockIdx.x * WAVES + wave; u < total; u += (int64_t)gridDim.x * WAVES) {
    const int s = segmented ? wave_find_segment(m.seg.group_prefix, m.seg.nseg, u) : 0;
    const int64_t tr = segmented ? u - m.seg.group_prefix[s] : u;  // row group in the segment
    const Segment g = load_segment(m.seg, s);
    if (!g.ok) continue;
    const int64_t r0 = tr * kGroupRows;
    const int nr = (int)min((int64_t)kGroupRows, g.na - r0);
    // the tile rows that cover the group (several when tiles are shorter
    // than the group, part of one when taller: entries of its other rows are
    // skipped below); their tiles are consecutive, so are their entries
    const int rlog = m.seg.rows_log2;
    const int64_t nct = col_tiles_of(g, rlog);
    const int64_t tbase = segmented ? m.seg.tile_prefix[s] : 0;
    const int64_t t0 = tbase + (r0 >> rlog) * nct;
    const int64_t t1 = tbase + (((r0 + nr - 1) >> rlog) + 1) * nct - 1;
    const bool have = t1 < m.tile_capacity;
    const int64_t e_begin = have ? m.tile_start[t0] : 0;
    const int64_t e_end = have ? m.tile_start[t1] + m.tile_count[t1] : 0;
    float2 acc[NACC];
#pragma unroll
    for (int j = 0; j < NACC; ++j) acc[j] = make_float2(0.f, 0.f);
    // one entry: its row in the group and the row box's gradient in gv
    // (every slot written), or -1 (gv untouched)
    auto entry = [&](int64_t e, float2 (&gv)[H]) -> int {
      if (e < 0 || e >= e_end || e >= m.capacity) return -1;
      // the entry's saved state in one round of loads (none waits for another)
      const int nx = m.s_nx[e];
      const int64_t pid = m.pair_id[e];
      const uint8_t* row = m.s_flags + e * (int64_t)m.cap;
      uint32_t codes[K / 2];
      if (m.flags_vec) {
        if constexpr (K == 4) {
          const uint2 w = *reinterpret_cast<const uint2*>(row);
          codes[0] = w.x;
          codes[1] = w.y;
        } else {
          const uint4 w = *reinterpret_cast<const uint4*>(row);
          codes[0] = w.x;
          codes[1] = w.y;
          codes[2] = w.z;
          codes[3] = w.w;
        }
      } else {
#pragma unroll
        for (int w = 0; w < K / 2; ++w) codes[w] = 0xffffffffu;
#pragma unroll
        for (int k = 0; k < CAP; ++k) {
          if (k < m.cap) {
            const uint32_t cc = row[k];
            codes[k >> 2] = (codes[k >> 2] & ~(0xffu << ((k & 3) * 8))) | (cc << ((k & 3) * 8));
          }
        }
      }
      if (nx == 0) return -1;  // empty intersection: zero gradient
      const int64_t local = pid - g.out0;
      if (local < 0 || g.nb <= 0) return -1;
      int64_t rg, col;  // row and column within the segment
      divmod(local, g.nb, rg, col);
      const int rl = (int)(rg - r0);
      if (rl < 0 || rl >= nr) return -1;
      int64_t ia = g.a0 + rg, ib = g.b0 + col;
      // self pairs: an entry below the diagonal was evaluated with the
      // column's box as P (the lower index), so the row's box is Q there
      const bool swapped = m.seg.self_pairs && rg > col;
      if (swapped) {
        const int64_t t = ia;
        ia = ib;
        ib = t;
      }
      const int n1 = FIXED ? K : poly_count(m.a.nv, ia, m.a.kmax);
      const int n2 = FIXED ? K : poly_count(m.b.nv, ib, m.b.kmax);
      Poly<K> P, Q;
      load_poly<K, FIXED>(m.a.xy, ia, m.a.kmax, m.a.vec4, n1, P);
      load_poly<K, FIXED>(m.b.xy, ib, m.b.kmax, m.b.vec4, n2, Q);
      // self pairs: entries (i, k) and (k, i) are one unordered pair with
      // one structure, so the row's box takes its role's gradient of that
      // pair weighted by both entries' upstream gradients
      float gw = m.grad[pid];
      if (m.seg.self_pairs) gw += m.grad[g.out0 + col * g.nb + rg];
      float lo1 = 0.f, hi1 = 0.f, lo2 = 0.f, hi2 = 0.f;
      if (Z3) {
        lo1 = m.a.zlo[ia];
        hi1 = m.a.zhi[ia];
        lo2 = m.b.zlo[ib];
        hi2 = m.b.zhi[ib];
      }
      float2 gP[K], gQ[K], gz1, gz2;
      bool thin;
      pair_backward<K, FIXED, Z3, BLOCK>(P, n1, Q, n2, gw, nx, codes, lo1, hi1, lo2, hi2,
                                         s_v + tid, s_g + tid, s_tab, gP, gQ, gz1, gz2, thin);
      if (thin) {  // rare: the gradient again in fp64, from the polygons reloaded
        load_poly<K, FIXED>(m.a.xy, opaque(ia), m.a.kmax, m.a.vec4, n1, P);
        load_poly<K, FIXED>(m.b.xy, opaque(ib), m.b.kmax, m.b.vec4, n2, Q);
        stage_pair<K, BLOCK>(s_v + tid, P, Q);
        pair_backward64<K, FIXED, Z3, BLOCK>(n1, n2, gw, nx, codes, lo1, hi1, lo2, hi2,
                                             s_v + tid, s_g + tid, gP, gQ, gz1, gz2);
      }
      const int nr_own = swapped ? n2 : n1;  // the row box's vertex count
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const bool own = FIXED || k < nr_own;  // padded slots: 0
        gv[k] = own ? (swapped ? gQ[k] : gP[k]) : make_float2(0.f, 0.f);
      }
      if constexpr (Z3) gv[K] = swapped ? gz2 : gz1;
      if (!m.seg.self_pairs) {
        float* ob = m.gb_xy + ib * (int64_t)m.b.kmax * 2;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if ((FIXED || k < n2) && k < m.b.kmax) {
            unsafeAtomicAdd(ob + 2 * k, gQ[k].x);
            unsafeAtomicAdd(ob + 2 * k + 1, gQ[k].y);
          }
        }
        if (Z3) {
          unsafeAtomicAdd(m.gb_z + 2 * ib, gz2.x);
          unsafeAtomicAdd(m.gb_z + 2 * ib + 1, gz2.y);
        }
      }
      return rl;
    };
    for (int64_t e0 = e_begin; e0 < e_end; e0 += 64) {  // uniform: every lane sums
      float2 gv[H];  // read only where rl >= 0
      const int rl = entry(e0 + lane, gv);
      step_row_sums<H, BLOCK>(rl, gv, stage, acc);
    }
    // each row of a belongs to exactly one row group: plain stores
#pragma unroll
    for (int j = 0; j < NACC; ++j) {
      const int c = lane + 64 * j;
      const int r = c / H, h = c - r * H;
      if (r < nr) {
        const int64_t ia = g.a0 + r0 + r;
        if (h < K) {
          if (h < kx) {
            m.ga_xy[(ia * kx + h) * 2] = acc[j].x;
            m.ga_xy[(ia * kx + h) * 2 + 1] = acc[j].y;
          }
        } else if (Z3) {
          m.ga_z[ia * 2] = acc[j].x;
          m.ga_z[ia * 2 + 1] = acc[j].y;
        }
      }
    }
  }
}

namespace {

template <bool B>
using Bool = std::integral_constant<bool, B>;

// Calls f(K, FIXED, Z3) with compile-time constants.
template <typename F>
void dispatch(int K, bool fixed, bool z3, F&& f) {
  auto go = [&](auto k, auto fx) {
    if (z3) f(k, fx, Bool<true>{}); else f(k, fx, Bool<false>{});
  };
  if (K == 4) {
    if (fixed) go(std::integral_constant<int, 4>{}, Bool<true>{});
    else go(std::integral_constant<int, 4>{}, Bool<false>{});
  } else {
    if (fixed) go(std::integral_constant<int, 8>{}, Bool<true>{});
    else go(std::integral_constant<int, 8>{}, Bool<false>{});
  }
}

bool valid_saved(const dgal_saved* s) {
  return s != nullptr && s->pair_id && s->nx && s->xflags && s->count && s->capacity >= 0 &&
         s->tile_start && s->tile_count && s->tile_mask && s->tile_capacity >= 0;
}

void zero(float* p, int64_t n, hipStream_t stream, Profiler* prof) {
  if (p != nullptr && n > 0) {
    const int64_t blocks = (n + 255) / 256;
    prof_begin(prof, stream);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)(blocks > 4096 ? 4096 : blocks)), dim3(256), 0,
                       stream, p, n);
    prof_end(prof, "k_fill_zero", stream);
  }
}

// Common validation of the matrix shapes; fills the segment arguments.
int check_shapes(dgal_polys a, dgal_polys b, const int64_t* a_off, const int64_t* b_off,
                 const int64_t* out_off, int nseg, int self_pairs, int64_t out_size,
                 const dgal_saved* saved, SegArgs& sa) {
  if (!valid_polys(a) || !valid_polys(b) || out_size < 0) return DGAL_EINVAL;
  if ((a.zlo == nullptr) != (b.zlo == nullptr)) return DGAL_EINVAL;
  const bool segmented = a_off != nullptr;
  if (segmented != (b_off != nullptr) || segmented != (out_off != nullptr)) return DGAL_EINVAL;
  if (segmented && (nseg < 1 || nseg > kMaxSeg)) return DGAL_EINVAL;
  if (self_pairs && !same_polys(a, b)) return DGAL_EINVAL;
  if (!segmented && (b.count >= (1 << 24) ||
                     (a.count > 0 && b.count > 0 && out_size / a.count < b.count)))
    return DGAL_EINVAL;
  if (!valid_saved(saved)) return DGAL_EINVAL;
  if (saved->tile_capacity > kScanTotals * (int64_t)kScanChunk) return DGAL_EINVAL;
  sa.a_off = a_off;
  sa.b_off = b_off;
  sa.out_off = out_off;
  sa.nseg = segmented ? nseg : 1;
  sa.a_count = a.count;
  sa.b_count = b.count;
  sa.out_size = out_size;
  sa.self_pairs = self_pairs;
  sa.tile_prefix = nullptr;
  sa.group_prefix = nullptr;
  sa.rows_log2 = 3;
  return DGAL_OK;
}

int64_t ceil_div(int64_t x, int64_t y) { return (x + y - 1) / y; }

}  // namespace

int matrix_forward(const CtxView& ctx, dgal_polys a, dgal_polys b, const int64_t* a_off,
                   const int64_t* b_off, const int64_t* out_off, int nseg, int self_pairs,
                   float* iou, int64_t out_size, dgal_saved* saved, hipStream_t stream,
                   const LaunchShape& shape) {
  SegArgs sa;
  const int st = check_shapes(a, b, a_off, b_off, out_off, nseg, self_pairs, out_size, saved, sa);
  if (st != DGAL_OK) return st;
  if (out_size > 0 && iou == nullptr) return DGAL_EINVAL;
  // the tile shape: the launch shape's, else the caller's, else the default
  const int R = shape.tile_rows > 0 ? shape.tile_rows
                : (saved->tile_rows > 0 ? saved->tile_rows : DGAL_TILE_ROWS_DEFAULT);
  sa.rows_log2 = tile_rows_log2(R);
  if (sa.rows_log2 < 0) return DGAL_EINVAL;
  saved->tile_rows = R;
  DeviceGuard dg(ctx.device);
  if (!dg.ok) return DGAL_EHIP;
  const int K = reg_k(a.kmax, b.kmax);
  const bool segmented = a_off != nullptr;
  int64_t single_tiles = 0;
  if (segmented) {
    // in the caller's saved state when it has room, for the backward
    int64_t* pre = saved->seg_prefix != nullptr ? saved->seg_prefix : ctx.prefix;
    sa.tile_prefix = pre;
    sa.group_prefix = pre + (kMaxSeg + 1);
    prof_begin(ctx.prof, stream);
    hipLaunchKernelGGL(k_seg_prep, dim3(1), dim3(256), 0, stream, sa, ctx.err, pre,
                       pre + (kMaxSeg + 1));
    prof_end(ctx.prof, "k_seg_prep", stream);
  } else {
    if (a.count == 0 || b.count == 0) return hipGetLastError() == hipSuccess ? DGAL_OK : DGAL_EHIP;
    single_tiles = ceil_div(a.count, R) * ceil_div(b.count, kTilePairs / R);
  }
  CullArgs c;
  c.seg = sa;
  c.a = poly_args(a, K);
  c.b = poly_args(b, K);
  c.single_tiles = single_tiles;
  c.iou = iou;
  c.pair_id = saved->pair_id;
  c.capacity = saved->capacity;
  c.tile_start = saved->tile_start;
  c.tile_count = saved->tile_count;
  c.tile_capacity = saved->tile_capacity;
  c.tile_mask = saved->tile_mask;
  c.err = ctx.err;
  ExactArgs x;
  x.seg = sa;
  x.a = c.a;
  x.b = c.b;
  x.iou = iou;
  x.pair_id = saved->pair_id;
  x.s_nx = saved->nx;
  x.s_flags = saved->xflags;
  x.capacity = saved->capacity;
  x.count = saved->count;
  x.cap = a.kmax + b.kmax;
  x.err = ctx.err;
  x.stats = ctx.stats;
  // 32 workgroups per CU by default: ranges of one or two tiles a wavefront
  // (c5: 110 us at 32, 48 or 64, 116 us at 16); a single block is capped below
  int64_t cull_grid = (int64_t)ctx.cus * (shape.cull_mult > 0 ? shape.cull_mult : 32);
  if (!segmented) cull_grid = std::min(cull_grid, ceil_div(single_tiles, kCullBlock / 64));
  const int exact_grid = ctx.cus * (shape.exact_mult > 0 ? shape.exact_mult : 8);
  const bool fixed = a.nv == nullptr && b.nv == nullptr && a.kmax == K && b.kmax == K &&
                     aligned(a.xy, 16) && aligned(b.xy, 16);
  dispatch(K, fixed, a.zlo != nullptr, [&](auto k, auto fx, auto z) {
    constexpr int KK = decltype(k)::value;
    constexpr bool FX = decltype(fx)::value, ZZ = decltype(z)::value;
    prof_begin(ctx.prof, stream);
    const dim3 cg((unsigned)cull_grid), cb(kCullBlock);
    if (R == 4) hipLaunchKernelGGL((k_matrix_cull<KK, FX, ZZ, 4>), cg, cb, 0, stream, c);
    else if (R == 16) hipLaunchKernelGGL((k_matrix_cull<KK, FX, ZZ, 16>), cg, cb, 0, stream, c);
    else hipLaunchKernelGGL((k_matrix_cull<KK, FX, ZZ, 8>), cg, cb, 0, stream, c);
    prof_end(ctx.prof, "k_matrix_cull", stream);
    if (saved->tile_capacity <= kScanSmall) {  // few tiles: one launch
      prof_begin(ctx.prof, stream);
      hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kScanBlock), 0, stream, sa.tile_prefix,
                         sa.nseg, single_tiles, saved->tile_capacity, saved->tile_start,
                         saved->tile_count, saved->count, saved->capacity, ctx.err);
      prof_end(ctx.prof, "k_scan_small", stream);
    } else {
      const int64_t chunks = std::max<int64_t>(1, ceil_div(saved->tile_capacity, kScanChunk));
      prof_begin(ctx.prof, stream);
      hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)chunks), dim3(kScanBlock), 0, stream,
                         sa.tile_prefix, sa.nseg, single_tiles, saved->tile_capacity,
                         saved->tile_count, ctx.scan);
      prof_end(ctx.prof, "k_scan_totals", stream);
      prof_begin(ctx.prof, stream);
      hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)chunks), dim3(kScanBlock), 0, stream,
                         sa.tile_prefix, sa.nseg, single_tiles, saved->tile_capacity, ctx.scan,
                         saved->tile_start, saved->tile_count, saved->count, saved->capacity,
                         ctx.err);
      prof_end(ctx.prof, "k_scan_apply", stream);
    }
    // the fill walks ~8 resident waves per SIMD, each over a contiguous range of tiles
    prof_begin(ctx.prof, stream);
    hipLaunchKernelGGL(k_matrix_fill, dim3((unsigned)std::max<int64_t>(1, (int64_t)ctx.cus * 8)),
                       dim3(kCullBlock), 0, stream, c);
    prof_end(ctx.prof, "k_matrix_fill", stream);
    prof_begin(ctx.prof, stream);
    hipLaunchKernelGGL((k_matrix_exact<KK, FX, ZZ>), dim3(exact_grid), dim3(kExactBlock), 0,
                       stream, x);
    prof_end(ctx.prof, "k_matrix_exact", stream);
  });
  return hipGetLastError() == hipSuccess ? DGAL_OK : DGAL_EHIP;
}

int matrix_backward(const CtxView& ctx, dgal_polys a, dgal_polys b, const int64_t* a_off,
                    const int64_t* b_off, const int64_t* out_off, int nseg, int self_pairs,
                    const float* grad_iou, int64_t out_size, const dgal_saved* saved,
                    float* grad_a_xy, float* grad_b_xy, float* grad_a_z, float* grad_b_z,
                    hipStream_t stream, const LaunchShape& shape) {
  SegArgs sa;
  const int st = check_shapes(a, b, a_off, b_off, out_off, nseg, self_pairs, out_size, saved, sa);
  if (st != DGAL_OK) return st;
  const bool z3 = a.zlo != nullptr;
  if (grad_iou == nullptr || grad_a_xy == nullptr) return DGAL_EINVAL;
  if (self_pairs ? (grad_b_xy != nullptr || grad_b_z != nullptr) : (grad_b_xy == nullptr))
    return DGAL_EINVAL;
  if (z3 != (grad_a_z != nullptr)) return DGAL_EINVAL;
  if (!self_pairs && z3 != (grad_b_z != nullptr)) return DGAL_EINVAL;
  sa.rows_log2 = tile_rows_log2(saved->tile_rows);  // the shape the forward recorded
  if (sa.rows_log2 < 0) return DGAL_EINVAL;
  DeviceGuard dg(ctx.device);
  if (!dg.ok) return DGAL_EHIP;
  const int K = reg_k(a.kmax, b.kmax);
  const bool segmented = a_off != nullptr;
  // every row of a is written by its row group, or zeroed by the kernel when
  // no row group holds it (segmented); without segments an empty b leaves no
  // row group at all.  Columns of a second set take atomic adds: zeroed
  // first.
  if (!segmented && b.count == 0) {
    zero(grad_a_xy, a.count * a.kmax * 2, stream, ctx.prof);
    if (z3) zero(grad_a_z, a.count * 2, stream, ctx.prof);
  }
  if (!self_pairs) {
    zero(grad_b_xy, b.count * b.kmax * 2, stream, ctx.prof);
    if (z3) zero(grad_b_z, b.count * 2, stream, ctx.prof);
  }
  int64_t single_groups = 0;
  if (segmented) {
    if (saved->seg_prefix != nullptr) {  // the forward's, kept with its work list
      sa.tile_prefix = saved->seg_prefix;
      sa.group_prefix = saved->seg_prefix + (kMaxSeg + 1);
    } else {
      // recomputed: another matrix call may have used the workspace since the forward
      sa.tile_prefix = ctx.prefix;
      sa.group_prefix = ctx.prefix + (kMaxSeg + 1);
      prof_begin(ctx.prof, stream);
      hipLaunchKernelGGL(k_seg_prep, dim3(1), dim3(256), 0, stream, sa, ctx.err, ctx.prefix,
                         ctx.prefix + (kMaxSeg + 1));
      prof_end(ctx.prof, "k_seg_prep", stream);
    }
  } else {
    if (a.count == 0 || b.count == 0) return hipGetLastError() == hipSuccess ? DGAL_OK : DGAL_EHIP;
    single_groups = ceil_div(a.count, kGroupRows);
  }
  BwdArgs m;
  m.seg = sa;
  m.a = poly_args(a, K);
  m.b = poly_args(b, K);
  m.single_groups = single_groups;
  m.grad = grad_iou;
  m.pair_id = saved->pair_id;
  m.s_nx = saved->nx;
  m.s_flags = saved->xflags;
  m.flags_vec = a.kmax + b.kmax == 2 * reg_k(a.kmax, b.kmax) &&
                aligned(saved->xflags, (uintptr_t)(a.kmax + b.kmax));
  m.capacity = saved->capacity;
  m.tile_start = saved->tile_start;
  m.tile_count = saved->tile_count;
  m.tile_capacity = saved->tile_capacity;
  m.cap = a.kmax + b.kmax;
  m.ga_xy = grad_a_xy;
  m.gb_xy = grad_b_xy;
  m.ga_z = grad_a_z;
  m.gb_z = grad_b_z;
  const bool fixed = a.nv == nullptr && b.nv == nullptr && a.kmax == K && b.kmax == K &&
                     aligned(a.xy, 16) && aligned(b.xy, 16);
  dispatch(K, fixed, z3, [&](auto k, auto fx, auto z) {
    constexpr int KK = decltype(k)::value;
    constexpr bool FX = decltype(fx)::value, ZZ = decltype(z)::value;
    int64_t grid = (int64_t)ctx.cus * (shape.bwd_mult > 0 ? shape.bwd_mult : 8);
    if (!segmented) grid = std::min(grid, ceil_div(single_groups, bwd_block<KK>() / 64));
    prof_begin(ctx.prof, stream);
    hipLaunchKernelGGL((k_matrix_bwd<KK, FX, ZZ>), dim3((unsigned)grid), dim3(bwd_block<KK>()), 0,
                       stream, m);
    prof_end(ctx.prof, "k_matrix_bwd", stream);
  });
  return hipGetLastError() == hipSuccess ? DGAL_OK : DGAL_EHIP;
}


// ---- scratch of the allocation-free forward (dgal_iou_matrix_noalloc) ----
// The work list, tile state, segment prefixes and scan totals that
// dgal_iou_matrix takes from the caller's dgal_saved and the context live
// here instead, in one static device array per GPU (allocated when the
// library's code object is loaded on that GPU, held until the process ends).
// Every call on a GPU shares its array: two such calls that overlap on one
// GPU race.  Nothing in it must start at zero (the forward writes every
// field it later reads, including the survivor count).
constexpr int64_t kNaTiles = DGAL_NOALLOC_MAX_TILES;
constexpr int64_t kNaPairs = DGAL_NOALLOC_MAX_PAIRS;
constexpr int64_t kNaFlags = 16;  // codes per entry: kmax_a + kmax_b <= 16
constexpr int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }
constexpr int64_t kNaPrefix = 0;  // int64 [2][DGAL_MAX_SEGMENTS + 1]
constexpr int64_t kNaScan = align256(kNaPrefix + 8 * 2 * (DGAL_MAX_SEGMENTS + 1));
constexpr int64_t kNaCount = align256(kNaScan + 8 * kScanTotals);
constexpr int64_t kNaTileStart = align256(kNaCount + 8);
constexpr int64_t kNaTileCount = align256(kNaTileStart + 8 * kNaTiles);
constexpr int64_t kNaTileMask = align256(kNaTileCount + 4 * kNaTiles);
constexpr int64_t kNaPairId = align256(kNaTileMask + 8 * kMaskWords * kNaTiles);
constexpr int64_t kNaNx = align256(kNaPairId + 8 * kNaPairs);
constexpr int64_t kNaXflags = align256(kNaNx + kNaPairs);
constexpr int64_t kNaBytes = align256(kNaXflags + kNaFlags * kNaPairs);
static_assert(kNaBytes == DGAL_NOALLOC_SCRATCH_BYTES, "scratch size stated in dgal.h");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {
constexpr int kNaDevices = 64;
std::mutex na_mu;
void* na_ptr[kNaDevices] = {};  // device address of `scratch` per GPU
}  // namespace

// Takes the device address of `scratch` on `device` (which must be current)
// once; later calls for the same device return at once.
int matrix_scratch_init(int device) {
  if (device < 0 || device >= kNaDevices) return DGAL_EINVAL;
  std::lock_guard<std::mutex> lock(na_mu);
  if (na_ptr[device] != nullptr) return DGAL_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
    return DGAL_EHIP;
  na_ptr[device] = ptr;
  return DGAL_OK;
}

int matrix_forward_noalloc(const CtxView& ctx, dgal_polys a, dgal_polys b, const int64_t* a_off,
                           const int64_t* b_off, const int64_t* out_off, int nseg,
                           int self_pairs, float* iou, int64_t out_size, hipStream_t stream,
                           const LaunchShape& shape) {
  void* base_v = nullptr;
  if (ctx.device >= 0 && ctx.device < kNaDevices) {
    std::lock_guard<std::mutex> lock(na_mu);
    base_v = na_ptr[ctx.device];
  }
  if (base_v == nullptr) return DGAL_EHIP;  // the context did not set this device up
  // one block: its tile count is known here, and a block past the scratch's
  // tiles is refused before anything is enqueued
  const int R = shape.tile_rows > 0 ? shape.tile_rows : DGAL_TILE_ROWS_DEFAULT;
  if (tile_rows_log2(R) < 0) return DGAL_EINVAL;
  if (a_off == nullptr && a.count > 0 && b.count > 0 &&
      ceil_div(a.count, R) > kNaTiles / ceil_div(b.count, kTilePairs / R))
    return DGAL_ECAPACITY;
  unsigned char* base = static_cast<unsigned char*>(base_v);
  dgal_saved sv;
  sv.pair_id = reinterpret_cast<int64_t*>(base + kNaPairId);
  sv.nx = base + kNaNx;
  sv.xflags = base + kNaXflags;
  sv.capacity = kNaPairs;
  sv.count = reinterpret_cast<int64_t*>(base + kNaCount);
  sv.tile_start = reinterpret_cast<int64_t*>(base + kNaTileStart);
  sv.tile_count = reinterpret_cast<int32_t*>(base + kNaTileCount);
  sv.tile_capacity = kNaTiles;
  sv.tile_mask = reinterpret_cast<uint64_t*>(base + kNaTileMask);
  sv.tile_rows = R;
  sv.seg_prefix = nullptr;  // the scratch's own prefixes
  CtxView v = ctx;
  v.prefix = reinterpret_cast<int64_t*>(base + kNaPrefix);
  v.scan = reinterpret_cast<int64_t*>(base + kNaScan);
  return matrix_forward(v, a, b, a_off, b_off, out_off, nseg, self_pairs, iou, out_size, &sv,
                        stream, shape);
}

}  // namespace dgal
