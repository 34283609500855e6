/*
 * dgal.h -- C ABI of the MI355X (gfx950) library for batched, differentiable
 * convex-polygon intersection-over-union.
 *
 * Paper: Y. Zhong, "Differentiable Computational Geometry for 2D and 3D machine
 * learning", arXiv 2011.11134.  Its Sec. II-B listing defines the operation:
 * the IoU of two convex polygons is the area of their intersection over
 * area(p1) + area(p2) - area(intersection); the forward keeps the number of
 * intersection vertices (nx) and one provenance flag per intersection vertex
 * (xflags), and the gradient is computed from the two polygons, the upstream
 * gradient, nx and xflags.  Sec. III fixes the data: polygons are convex,
 * counter-clockwise, stored in fixed-capacity vertex arrays, and gradients are
 * stored in the same polygon layout.  Sec. IV-A applies it to rotated 2D and
 * 3D boxes.
 *
 * Conventions for every entry point:
 *   - Every data pointer is CALLER-OWNED DEVICE memory on the context's device.
 *     Nothing is retained after the call returns.
 *   - Work is enqueued on `stream` (a hipStream_t, passed as void*; NULL is the
 *     null stream) and runs asynchronously.  Outputs are OVERWRITTEN.
 *   - The library allocates no memory per call; its only allocations are made
 *     by dgal_create (a small workspace) and freed by dgal_destroy.
 *   - Returns DGAL_OK (0) or a negative status.  Arguments are validated on the
 *     host before anything is enqueued; on error nothing is enqueued.  No C++
 *     exception crosses this interface.
 *   - Per-element data (vertex counts outside [3, kmax], clockwise or
 *     non-convex polygons) is not validated on the fast path: results for
 *     such elements are unspecified, but every memory access stays in
 *     bounds.  dgal_validate checks it, and dgal_set_validate (or
 *     DGAL_DEBUG_VALIDATE=1) turns the check on before every call.  An intersection
 *     that would overflow its capacity (possible only for invalid polygons)
 *     sets a sticky device error that dgal_check reports as DGAL_ECAPACITY.
 *   - A context may be used from one host thread at a time.
 *
 * Polygon layout (Sec. III): xy is [count][kmax][2] fp32 (x, y interleaved),
 * vertices counter-clockwise and strictly convex, slots >= nv[i] ignored;
 * the base pointer must be 8-byte aligned.  Intersections hold at most
 * kmax_a + kmax_b vertices.
 *
 * Provenance codes (one uint8 per intersection vertex, listed counter-
 * clockwise starting at the smallest code; unused slots hold 0xFF):
 *   vertex i of polygon a             -> i               (0x00..0x07)
 *   vertex j of polygon b             -> 0x10 | j        (0x10..0x17)
 *   edge i of a crossing edge j of b  -> 0x40 | i<<3 | j (0x40..0x7F)
 * Edge i runs from vertex i to vertex (i+1) mod n.
 *
 * Degenerate contacts (a vertex exactly on an edge line, collinear edges,
 * identical polygons) are resolved as if polygon b were moved by
 * (eps, eps^2), eps -> 0+; exact zeros of the orientation test take the sign
 * of that motion.  Orientation signs are certified in fp32 and recomputed in
 * fp64 (exactly, for fp32 inputs) when fp32 cannot certify them.
 */
#ifndef DGAL_H
#define DGAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DGAL_OK = 0,
  DGAL_EINVAL = -1,    /* invalid argument (see each entry point) */
  DGAL_ECAPACITY = -2, /* deferred: an intersection or a saved-pair list overflowed */
  DGAL_EHIP = -3,      /* HIP runtime or launch error */
  DGAL_EIO = -4        /* a file could not be read or written (tune cache) */
};

typedef struct dgal_ctx dgal_ctx;

/* A set of polygons (Sec. III), optionally with a z-extent for 3D boxes. */
typedef struct {
  const float *xy;     /* [count][kmax][2] fp32, 8-byte aligned                  */
  const uint8_t *nv;   /* [count] vertex counts in [3, kmax]; NULL => all kmax     */
  const float *zlo;    /* [count] bottom of the z-extent, or NULL for 2D          */
  const float *zhi;    /* [count] top of the z-extent, or NULL for 2D             */
  int64_t count;       /* number of polygons, >= 0                                */
  int32_t kmax;        /* vertex capacity, 3..8                                   */
} dgal_polys;

/* Creates a context on HIP device `hip_device` (allocates a small device
 * workspace).  *out is set to NULL on failure.  Returns DGAL_OK, DGAL_EINVAL
 * (out == NULL) or DGAL_EHIP. */
int dgal_create(dgal_ctx **out, int hip_device);

/* Frees the context and its workspace; NULL is a no-op.  The caller must make
 * sure no work enqueued with the context is still running. */
void dgal_destroy(dgal_ctx *ctx);

/* Static string for a status code. */
const char *dgal_status_string(int status);

/* Synchronises `stream`, then returns (and clears) any sticky device-side
 * error: DGAL_ECAPACITY (an overflow), DGAL_EINVAL (segment offsets the
 * kernels rejected), DGAL_EHIP for a runtime error, else DGAL_OK. */
int dgal_check(dgal_ctx *ctx, void *stream);

/* Sec. II-B listing, batched: iou[i] = IoU(a[i], b[i]) for i < a.count.
 * 3D (all four z pointers non-NULL): BEV intersection area times the
 * z-overlap, over the union volume (Sec. IV-A "3D IoU").
 *   iou    [count] fp32
 *   nx     [count] uint8 intersection vertex counts        } saved for the
 *   xflags [count][a.kmax + b.kmax] uint8 provenance codes } backward; both
 *          NULL => forward only.
 * DGAL_EINVAL: ctx/iou/a.xy/b.xy NULL with count > 0, count < 0, a.count !=
 * b.count, kmax outside 3..8, exactly one of nx/xflags NULL, z pointers given
 * for only one of a/b or only one of zlo/zhi, misaligned xy. */
int dgal_iou_pairs(dgal_ctx *ctx, dgal_polys a, dgal_polys b, float *iou,
                   uint8_t *nx, uint8_t *xflags, void *stream);

/* The matrix kernels work in tiles of DGAL_TILE_PAIRS pairs of one block:
 * tile_rows rows x DGAL_TILE_PAIRS / tile_rows columns, with tile_rows 4, 8
 * or 16 (512, 256 or 128 columns), chosen per call (dgal_saved.tile_rows). */
#define DGAL_TILE_PAIRS 2048
#define DGAL_TILE_ROWS_DEFAULT 8

/* Work list and saved state of a matrix forward: one entry per pair that
 * survived the conservative cull (every other pair is disjoint: its IoU is 0
 * and its gradient zero), with the intersection's vertex count and provenance
 * codes (nx == 0 for a survivor whose intersection is empty), and a table that
 * gives each tile its contiguous range of entries.  Tiles are numbered segment
 * by segment, row-major over the segment's tile grid (ceil(rows / tile_rows)
 * x ceil(cols / tile_cols) tiles per segment with both sides non-empty).  All
 * pointers are device memory; the forward overwrites everything, including
 * *count.  Entries are laid out tile by tile, in a fixed order. */
#define DGAL_TILE_MASK_WORDS (DGAL_TILE_PAIRS / 64 + 2)

typedef struct {
  int64_t *pair_id;       /* [capacity] index into the flat iou output               */
  uint8_t *nx;            /* [capacity]                                               */
  uint8_t *xflags;        /* [capacity][a.kmax + b.kmax]                              */
  int64_t capacity;       /* entries available; overflow => DGAL_ECAPACITY (deferred,
                             and the overflowing pairs' IoU is not written)           */
  int64_t *count;         /* device scalar: survivors found (may exceed capacity)    */
  int64_t *tile_start;    /* [tile_capacity] first entry of each tile                 */
  int32_t *tile_count;    /* [tile_capacity] entries of each tile                     */
  int64_t tile_capacity;  /* >= number of tiles, else DGAL_ECAPACITY (deferred)       */
  uint64_t *tile_mask;    /* [tile_capacity][DGAL_TILE_MASK_WORDS] per tile, written by
                             the forward: words 0..31 the survivor bits (word
                             c * tile_rows + r: row r, columns 64c .. 64c + 63
                             of the tile), word 32 the output index of the tile's
                             first element, word 33 its block's row length      */
  int32_t tile_rows;      /* HOST field, in/out.  In: 4, 8 or 16 fixes the tile
                             shape; 0 lets the forward choose it (the autotuned
                             shape of this kind of call, else
                             DGAL_TILE_ROWS_DEFAULT).  Out: the forward writes
                             the rows it used, which the backward reads.  With 0,
                             tile_capacity must hold the tiles of every shape
                             (the largest of the three counts).                   */
  int64_t *seg_prefix;    /* [2][DGAL_MAX_SEGMENTS + 1] or NULL (segmented calls):
                             the forward writes its segments' tile and row-group
                             prefixes here (else into the context's workspace),
                             and a backward given them does not recompute them
                             (they hold for the offsets and tile shape of the
                             forward that wrote them).                           */
} dgal_saved;

/* Most segments one matrix call may hold. */
#define DGAL_MAX_SEGMENTS 4096

/* IoU matrices (Sec. IV-A case study at scale), segmented.  For segment s,
 * rows a[a_off[s] .. a_off[s+1]) and columns b[b_off[s] .. b_off[s+1]) form a
 * row-major block of iou starting at element out_off[s].  With a_off ==
 * b_off == out_off == NULL (nseg ignored) there is one block a.count x b.count
 * at iou[0].  self_pairs != 0 means b is a (same pointers and counts; each
 * segment's block is square): the diagonal of each block is exactly 1, and
 * entries (r, c) and (c, r) are the IoU of one unordered pair, evaluated with
 * the lower-indexed polygon first (so the tie rule moves the higher-indexed
 * one, and z-overlap ties go to the lower-indexed one): the block is
 * symmetric and each pair has one derivative structure.
 *   a_off, b_off  DEVICE int64 [nseg+1], non-decreasing, within [0, count]
 *   out_off       DEVICE int64 [nseg]
 *   out_size      number of fp32 elements the caller allocated at iou
 *   iou           flat fp32 output; element indices are 64-bit, so an output
 *                 may hold more than 2^31 elements
 *   saved         REQUIRED: the forward's work list, also the state that
 *                 dgal_iou_backward needs (a forward-only caller may discard it);
 *                 its tile_rows chooses the tile shape and returns the one used.
 * Offsets live on the device so that the call can be captured in a HIP graph;
 * the kernels check them (a block outside [0, out_size) or rows/columns
 * outside [0, count) is skipped and reported by dgal_check as DGAL_EINVAL).
 * DGAL_EINVAL (immediate): as dgal_iou_pairs except a.count == b.count, plus
 * some but not all offsets NULL, nseg outside [1, DGAL_MAX_SEGMENTS] with
 * offsets, out_size < a.count * b.count without offsets, a block with 2^24 or
 * more columns, self_pairs with a and b differing, saved with a NULL field or
 * a negative capacity, saved NULL, saved->tile_rows not 0, 4, 8 or 16. */
int dgal_iou_matrix(dgal_ctx *ctx, dgal_polys a, dgal_polys b,
                    const int64_t *a_off, const int64_t *b_off,
                    const int64_t *out_off, int32_t nseg, int32_t self_pairs,
                    float *iou, int64_t out_size, dgal_saved *saved,
                    void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * forward of dgal_iou_matrix, with the same arguments less `saved`, whose
 * work list, tile state and workspace live in a static device array of the
 * library (DGAL_NOALLOC_SCRATCH_BYTES, held on each GPU the library runs on
 * until the process ends; its address is taken once per device by
 * dgal_create).  Nothing is allocated and nothing synchronises; the output is
 * the same as dgal_iou_matrix's for the same input.  Limits: at most
 * DGAL_NOALLOC_MAX_TILES tiles (ceil(rows / tile_rows) x ceil(cols /
 * tile_cols) per block, in the shape dgal_iou_matrix would use: the one the
 * autotuner chose for this kind of call, else DGAL_TILE_ROWS_DEFAULT rows)
 * and DGAL_NOALLOC_MAX_PAIRS pairs surviving the cull.  One block over the
 * tile limit returns DGAL_ECAPACITY before anything is enqueued; segments
 * (whose sizes are on the device) over either limit, and one block over the
 * survivor limit, are reported by dgal_check as DGAL_ECAPACITY, with the IoU
 * of the pairs past the limit not written.  All calls on one GPU share the
 * array: calls that overlap on one GPU (two streams, two host threads) race,
 * and the backward cannot follow this call (it keeps no state for the
 * caller).  DGAL_EINVAL: as dgal_iou_matrix, without the conditions on saved.
 * DGAL_EHIP: the context was not created on a device the scratch serves. */
#define DGAL_NOALLOC_MAX_TILES 65536
#define DGAL_NOALLOC_MAX_PAIRS 1048576
#define DGAL_NOALLOC_SCRATCH_BYTES 44925440 /* ~42.8 MiB */
int dgal_iou_matrix_noalloc(dgal_ctx *ctx, dgal_polys a, dgal_polys b,
                            const int64_t *a_off, const int64_t *b_off,
                            const int64_t *out_off, int32_t nseg, int32_t self_pairs,
                            float *iou, int64_t out_size, void *stream);

enum { DGAL_PAIRS = 0, DGAL_MATRIX = 1 };

/* Sec. II-B `iou_grad`: gradient of sum(grad_iou * iou) with respect to the
 * vertices (and z-extents) of a and b, from the saved state of the forward
 * (no intersection is recomputed from predicates).
 * mode DGAL_PAIRS:  grad_iou [count]; nx, xflags as written by dgal_iou_pairs;
 *                   saved and offsets ignored.
 * mode DGAL_MATRIX: grad_iou has the shape of the matrix output (out_size
 *                   elements, ignored in pairs mode); `saved` as
 *                   written by dgal_iou_matrix with the same a, b, offsets and
 *                   self_pairs; nx / xflags ignored.  With self_pairs the
 *                   gradient of both roles accumulates into grad_a_* and
 *                   grad_b_* must be NULL; the diagonal contributes nothing,
 *                   and each unordered pair's gradient (the lower index as
 *                   the first polygon) is weighted by the sum of its two
 *                   entries' upstream gradients.
 * Outputs (overwritten; padded vertex slots are written 0):
 *   grad_a_xy [a.count][a.kmax][2], grad_b_xy [b.count][b.kmax][2] fp32
 *   grad_a_z, grad_b_z [count][2] fp32 = (d/dzlo, d/dzhi); NULL for 2D.
 * The matrix mode sums each row's gradient in a fixed order (its entries in
 * work-list order) and writes every row once, so rows (and every self-pair
 * gradient) are the same bits from run to run; with two different sets the
 * column gradients are added with fp32 global atomics (their order, and so
 * the low-order bits, may vary).
 * The matrix mode reads the tile shape the forward recorded in
 * saved->tile_rows.
 * DGAL_EINVAL: as the forward, plus a NULL required output or saved state, an
 * unknown mode, z outputs requested for 2D input, saved->tile_rows not 4, 8
 * or 16. */
int dgal_iou_backward(dgal_ctx *ctx, int32_t mode, dgal_polys a, dgal_polys b,
                      const int64_t *a_off, const int64_t *b_off,
                      const int64_t *out_off, int32_t nseg, int32_t self_pairs,
                      const float *grad_iou, int64_t out_size, const uint8_t *nx,
                      const uint8_t *xflags, const dgal_saved *saved,
                      float *grad_a_xy, float *grad_b_xy, float *grad_a_z,
                      float *grad_b_z, void *stream);

/* The intersection primitive under the IoU (Sec. II-B: the convex polygon
 * P n Q with its vertex count and one provenance flag per vertex; Sec. III:
 * fixed-capacity storage), batched: for i < a.count,
 *   out_xy [count][a.kmax + b.kmax][2] fp32: the intersection's vertices,
 *          counter-clockwise from the smallest code, absolute coordinates;
 *          slots at and past nx[i] are written 0
 *   nx     [count] uint8, xflags [count][a.kmax + b.kmax] uint8 (0xFF padded):
 *          the same values dgal_iou_pairs saves.
 * All three outputs are required.  DGAL_EINVAL: as dgal_iou_pairs (z pointers
 * are ignored), plus a NULL output or out_xy not 8-byte aligned. */
int dgal_intersect(dgal_ctx *ctx, dgal_polys a, dgal_polys b, float *out_xy,
                   uint8_t *nx, uint8_t *xflags, void *stream);

/* Backward of dgal_intersect: the gradient of sum <grad_xy, out_xy> with
 * respect to the vertices of a and b, from the saved nx / xflags (each
 * vertex rebuilt from its code: a polygon vertex passes its gradient
 * through, a crossing takes the chain rule of the two edges' meeting point).
 *   grad_xy [count][a.kmax + b.kmax][2] fp32 (slots past nx are ignored)
 *   grad_a_xy [count][a.kmax][2], grad_b_xy [count][b.kmax][2] fp32,
 *   overwritten, padded slots written 0.
 * DGAL_EINVAL: as dgal_intersect, plus a NULL input or output. */
int dgal_intersect_backward(dgal_ctx *ctx, dgal_polys a, dgal_polys b,
                            const float *grad_xy, const uint8_t *nx,
                            const uint8_t *xflags, float *grad_a_xy,
                            float *grad_b_xy, void *stream);

/* Sec. III polygon area (shoelace about the first vertex; positive for a
 * counter-clockwise polygon), batched: area [p.count] fp32.  z ignored.
 * DGAL_EINVAL: ctx NULL, invalid p, area NULL with count > 0. */
int dgal_area(dgal_ctx *ctx, dgal_polys p, float *area, void *stream);

/* Backward of dgal_area: grad_xy [count][kmax][2] = grad_area[i] *
 * d area / d vertex, i.e. (y_next - y_prev, x_prev - x_next) / 2 times the
 * upstream gradient (cyclic neighbours; padded slots written 0). */
int dgal_area_backward(dgal_ctx *ctx, dgal_polys p, const float *grad_area,
                       float *grad_xy, void *stream);

/* IoU of SIMPLE polygons: counter-clockwise, not self-intersecting, not
 * necessarily convex (Sec. III keeps polygons convex and plans arbitrary
 * ones; Sec. V lists arbitrary shapes as future work).  Elementwise pairs,
 * 2D only.  The intersection area is half the boundary integral of
 * x dy - y dx (Green's theorem): each edge contributes the cross product of
 * its end points times the fraction of the edge inside the other polygon,
 * found from the edge's crossings with the other boundary and the inclusion
 * of its start vertex; no intersection polygon is formed.  Orientation signs
 * and degenerate contacts follow the same rules as the convex path.
 *   a, b: as for dgal_iou_pairs (kmax 3..8, counts optional), zlo/zhi NULL.
 *   iou [count] fp32, overwritten.
 *   Saved state for dgal_iou_simple_backward (all three NULL => forward
 *   only; otherwise all non-NULL), overwritten:
 *     xmask [count] uint64 (8-byte aligned): bit 8*i + j set when edge i of
 *       a crosses edge j of b (edge i runs from vertex i to vertex i+1 mod n);
 *     smask [count] uint64: the same bit set when, in addition, edge i of a
 *       enters b there (vertex i of a lies right of edge j of b);
 *     inside [count] uint8: bit 0 when vertex 0 of a is inside b, bit 1 when
 *       vertex 0 of b is inside a.
 * Self-intersecting or clockwise input is not detected on the fast path
 * (results unspecified, accesses in bounds); dgal_validate_simple checks it,
 * and with dgal_set_validate on, this entry point and its backward run that
 * check first.
 * DGAL_EINVAL: ctx NULL, invalid a or b, a.count != b.count, a z-extent
 * given, saved pointers partly NULL or misaligned, iou NULL with count > 0. */
int dgal_iou_simple_pairs(dgal_ctx *ctx, dgal_polys a, dgal_polys b, float *iou,
                          uint64_t *xmask, uint64_t *smask, uint8_t *inside,
                          void *stream);

/* Backward of dgal_iou_simple_pairs from its saved state: moving a vertex
 * moves its two edges, and the intersection area changes by each edge's
 * outward normal (dy, -dx) times the integral, over the edge's parts inside
 * the other polygon, of how far along the edge the point moves with the
 * vertex; the polygon areas by the shoelace formula; then the quotient rule
 * of IoU.
 *   grad_iou [count] fp32; xmask, smask, inside as saved by the forward.
 *   grad_a_xy [count][a.kmax][2], grad_b_xy [count][b.kmax][2] fp32 (8-byte
 *   aligned), overwritten, padded slots written 0.
 * DGAL_EINVAL: as the forward, plus a NULL or misaligned pointer. */
int dgal_iou_simple_backward(dgal_ctx *ctx, dgal_polys a, dgal_polys b,
                             const float *grad_iou, const uint64_t *xmask,
                             const uint64_t *smask, const uint8_t *inside,
                             float *grad_a_xy, float *grad_b_xy, void *stream);

/* The input contract of Sec. III, checked per polygon: the vertex count is
 * in [3, kmax], every turn v[k-1] -> v[k] -> v[k+1] is strictly left (the
 * orientation of the three fp32 vertices evaluated in fp64 as
 * (v[k] - v[k-1]) x (v[k+1] - v[k-1]) is > 0), and the boundary turns around
 * exactly once (a star polygon such as the pentagram turns left at every
 * vertex but winds twice).  z is ignored.
 *   status [p.count] uint8, overwritten (may be NULL): 0 valid, 1 vertex
 *     count out of range, 2 a turn not strictly left (clockwise order, a
 *     reflex, straight or repeated vertex), 3 winds more than once.
 *   n_bad: device int64 scalar (may be NULL), overwritten with the number of
 *     invalid polygons (zeroed by a kernel on the stream, so the call can be
 *     captured in a graph).
 * DGAL_EINVAL: ctx NULL, invalid p (as elsewhere), both outputs NULL, n_bad
 * not 8-byte aligned. */
int dgal_validate(dgal_ctx *ctx, dgal_polys p, uint8_t *status, int64_t *n_bad,
                  void *stream);

/* The simple-polygon contract of dgal_iou_simple_pairs, checked per polygon:
 * the vertex count is in [3, kmax]; no two non-adjacent edges touch or cross
 * (collinear edges that do not overlap are allowed) and no two adjacent
 * edges fold back onto each other; the shoelace area is positive
 * (counter-clockwise).  Every test is the fp64 sign of the fp32 vertices
 * evaluated in a fixed order.  status: 0 valid, 1 vertex count out of
 * range, 2 edges meet or overlap, 3 area not positive; n_bad and errors as
 * for dgal_validate. */
int dgal_validate_simple(dgal_ctx *ctx, dgal_polys p, uint8_t *status,
                         int64_t *n_bad, void *stream);

/* Input checking before every call (off by default; on at dgal_create when
 * the environment holds DGAL_DEBUG_VALIDATE=1).  While on, dgal_iou_pairs,
 * dgal_iou_matrix, dgal_iou_backward, dgal_intersect and
 * dgal_intersect_backward first run dgal_validate's check on their polygon
 * sets, wait for it on the stream, and return DGAL_EINVAL, enqueueing
 * nothing else, if any polygon breaks the contract.  A debugging aid: it
 * synchronises the stream, so calls must not be captured in a graph while
 * it is on.  dgal_area and its backward accept any simple polygon and are
 * not checked; dgal_iou_simple_pairs and its backward run the check of
 * dgal_validate_simple instead.  DGAL_EINVAL: ctx NULL. */
int dgal_set_validate(dgal_ctx *ctx, int32_t enable);

/* Path statistics (off by default; the numerical-stability question the
 * paper leaves open after Sec. II-C and in Sec. V).  While enabled, the
 * forward kernels of dgal_iou_pairs, dgal_iou_matrix (its exact pass),
 * dgal_intersect and dgal_iou_boxes count on the device the pairs they
 * evaluate, those whose orientation signs fp32 could not certify and
 * recomputed in fp64, and those whose areas were rebuilt in fp64 (thin
 * pairs: the pair's largest coordinate in the frame at its first polygon's
 * vertex 0, squared, above 32 times the union; dgal_intersect rebuilds
 * none), with one set of atomic adds per wavefront.  dgal_path_stats
 * synchronises `stream`, returns the three counts and clears them.
 * DGAL_EINVAL: ctx NULL (set), or ctx / an output NULL (read). */
int dgal_set_path_stats(dgal_ctx *ctx, int32_t enable);
int dgal_path_stats(dgal_ctx *ctx, int64_t *pairs, int64_t *fp64_pairs, int64_t *thin_pairs,
                    void *stream);

/* Launch-shape autotuning of the batched kernels: the grid of the pair
 * kernels; for the matrix forward, the tile shape (4, 8 or 16 rows, unless
 * saved->tile_rows fixes it) and the persistent grids of its count and exact
 * passes; the persistent grid of the matrix backward (Sec. II-C: kernels
 * specialised per size).  Kinds of call are told apart by entry point, vertex
 * capacity 4 or 8, fixed-size or counted polygons, 2D or 3D, one block or
 * segments, and a size bucket (the bit lengths of the counts).  A call of a
 * kind with no choice yet takes the process-wide store's (see
 * dgal_tune_cache_load), else, while tuning is enabled, times each candidate
 * on the caller's own buffers (two interleaved passes of one warm-up and
 * three timed runs, HIP events on the caller's stream, the faster pass
 * kept), drops any candidate that raises the sticky device error (a tile
 * table too small for its shape), keeps the fastest (the built-in shape
 * unless another beats it by more than 5%) in the context and in the store
 * (and in the DGAL_TUNE_CACHE file, if set), and produces its outputs with
 * one more run of it; later calls of that kind use the choice, enabled or
 * not.  That first call synchronises the stream (so it
 * must not be captured in a graph), creates two HIP events, and is skipped
 * (built-in shapes) while the device error word holds an earlier call's
 * error.  Disabled by default: built-in shapes.  DGAL_EINVAL: ctx NULL. */
int dgal_set_autotune(dgal_ctx *ctx, int32_t enable);

/* Writes one line per tuned kind of this context into buf ("<key>: grid=..
 * cull=.. exact=.. bwd=.. rows=..", NUL-terminated, truncated to size) and
 * returns the number of tuned kinds; DGAL_EINVAL for ctx NULL, a negative
 * size, or buf NULL with size > 0. */
int dgal_autotune_report(dgal_ctx *ctx, char *buf, int64_t size);

/* The process-wide store of tuned launch shapes, shared by every context and
 * keyed by "<gfx arch>/<kind>/K<4|8>/fixed<0|1>/z<0|1>/seg<0|1>/b<bucket>",
 * and its JSON file:
 *   {"format": "dgal-tune-cache", "version": 1, "entries": [{"key": "...",
 *    "grid": G, "cull_mult": C, "exact_mult": E, "bwd_mult": B,
 *    "tile_rows": R, "ms": T}, ...]}
 * If DGAL_TUNE_CACHE names a file when the first context is created, it is
 * loaded then, and rewritten (a temporary file renamed over it) after every
 * tuning; a file that exists but does not load as a cache is never written.
 * No GPU is needed for these four calls.
 * dgal_tune_cache_load merges a file's entries (a file entry replaces one of
 * the same key) and returns their number; DGAL_EIO if it cannot be read,
 * DGAL_EINVAL if path is NULL or the file is not a cache or holds a value
 * outside the launchable ranges (then nothing is merged).
 * dgal_tune_cache_save writes the store: DGAL_OK, DGAL_EIO, DGAL_EINVAL
 * (path NULL).  dgal_tune_cache_report writes one line per entry ("<key>
 * grid=.. cull=.. exact=.. bwd=.. rows=.. ms=..") into buf (NUL-terminated,
 * truncated to size) and returns the entry count (DGAL_EINVAL: a negative
 * size, or buf NULL with size > 0).  dgal_tune_cache_clear empties the store
 * (contexts keep the choices they already made). */
int dgal_tune_cache_load(const char *path);
int dgal_tune_cache_save(const char *path);
int dgal_tune_cache_report(char *buf, int64_t size);
int dgal_tune_cache_clear(void);

/* Per-kernel timing, a measuring aid (off by default).  While enabled, every
 * kernel the library launches is bracketed by two HIP events on the caller's
 * stream and waited for, and its duration is added to its kernel's total;
 * calls therefore synchronise and must not be captured in a graph.  Enabling
 * resets the totals.  DGAL_EINVAL: ctx NULL; DGAL_EHIP: event creation. */
int dgal_set_profiling(dgal_ctx *ctx, int32_t enable);

/* Writes one line per kernel timed since profiling was enabled,
 * "<kernel> <launches> <total milliseconds>", into buf (NUL-terminated,
 * truncated to size) and returns the number of kernels; DGAL_EINVAL for ctx
 * NULL, a negative size, or buf NULL with size > 0; DGAL_EHIP if an event
 * call failed while timing. */
int dgal_profile_report(dgal_ctx *ctx, char *buf, int64_t size);

/* Rotated boxes by their parameters (Sec. IV-A case study), the corners
 * formed in-kernel: corner k = (cx, cy) + R(yaw) (+-l/2, +-w/2),
 * counter-clockwise from (+l/2, -w/2), i.e. the length along the heading.
 *   p      [count][dim] fp32 rows: dim 5 = (cx, cy, w, l, yaw) for 2D,
 *          dim 7 = (cx, cy, w, l, yaw, z, h) for 3D (z the centre: the
 *          extent is [z - h/2, z + h/2]); rows 4-byte aligned. */
typedef struct {
  const float *p;
  int64_t count;
  int32_t dim;
} dgal_boxes;

/* IoU of box pairs (2D or 3D as the boxes' dim), batched like
 * dgal_iou_pairs: iou [count] fp32; nx [count] uint8 and xflags [count][8]
 * uint8 (8-byte aligned) saved for the backward, both NULL => forward only.
 * DGAL_EINVAL: ctx or p NULL with count > 0, count < 0, a.count != b.count,
 * dim not 5 / 7 or differing, iou NULL, exactly one of nx / xflags NULL,
 * misaligned xflags. */
int dgal_iou_boxes(dgal_ctx *ctx, dgal_boxes a, dgal_boxes b, float *iou,
                   uint8_t *nx, uint8_t *xflags, void *stream);

/* Gradient of sum(grad_iou * iou) with respect to the box parameters, from
 * the saved nx / xflags: the corner gradient of dgal_iou_backward carried
 * through the corner formula (and zlo = z - h/2, zhi = z + h/2).
 *   grad_a, grad_b [count][dim] fp32, overwritten.
 * DGAL_EINVAL: as dgal_iou_boxes, plus a NULL input or output. */
int dgal_iou_boxes_backward(dgal_ctx *ctx, dgal_boxes a, dgal_boxes b,
                            const float *grad_iou, const uint8_t *nx,
                            const uint8_t *xflags, float *grad_a, float *grad_b,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DGAL_H */
