// internal.hpp -- declarations shared by the C ABI (api.hip) and the kernel
// translation units.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dgal.h"
#include "tune_cache.hpp"

namespace dgal {

// Bits of the sticky device error word.
enum : int { kErrCapacity = 1, kErrSegment = 2 };

struct PolyArgs {
  const float* xy;
  const uint8_t* nv;
  const float* zlo;
  const float* zhi;
  int64_t count;
  int kmax;
  bool vec4;  // rows of exactly K vertices, 16-byte aligned
};

struct PairsFwdArgs {
  PolyArgs a, b;
  float* iou;
  uint8_t* nx;
  uint8_t* xflags;
  int cap;        // a.kmax + b.kmax: bytes per xflags row
  bool flags_vec; // cap == 2K and rows aligned to cap bytes
  int* err;
  unsigned long long* stats;  // path statistics (NULL: off)
};

struct PairsBwdArgs {
  PolyArgs a, b;
  const float* grad;
  const uint8_t* nx;
  const uint8_t* xflags;
  int cap;
  bool flags_vec;
  float* ga_xy;
  float* gb_xy;
  float* ga_z;
  float* gb_z;
};

struct IntersectArgs {
  PolyArgs a, b;
  float* out_xy;    // [count][cap][2]
  uint8_t* nx;
  uint8_t* xflags;  // [count][cap]
  int cap;          // a.kmax + b.kmax
  bool rows_vec;    // cap == 2K, vertex rows 16-byte and flag rows cap-byte aligned
  int* err;
  unsigned long long* stats;  // path statistics (NULL: off)
};

struct IntersectBwdArgs {
  PolyArgs a, b;
  const float* grad_xy;  // [count][cap][2]
  const uint8_t* nx;
  const uint8_t* xflags;
  int cap;
  bool rows_vec;  // cap == 2K; gradient rows and outputs 16-byte, flag rows cap-byte aligned
  float* ga_xy;
  float* gb_xy;
};

struct BoxesFwdArgs {
  const float* a;   // [count][5 or 7]
  const float* b;
  int64_t count;
  float* iou;
  uint8_t* nx;
  uint8_t* xflags;  // [count][8], 8-byte aligned
  int* err;
  unsigned long long* stats;  // path statistics (NULL: off)
};

struct BoxesBwdArgs {
  const float* a;
  const float* b;
  int64_t count;
  const float* grad;
  const uint8_t* nx;
  const uint8_t* xflags;
  float* ga;  // [count][5 or 7]
  float* gb;
};

// Simple (not necessarily convex) polygon pairs: IoU and the saved state
// (crossing mask, entering mask, vertex-0 inclusion bits).
struct SimpleFwdArgs {
  PolyArgs a, b;
  float* iou;
  uint64_t* xmask;  // NULL: forward only (then smask and inside are NULL too)
  uint64_t* smask;
  uint8_t* inside;
};

struct SimpleBwdArgs {
  PolyArgs a, b;
  const float* grad;
  const uint64_t* xmask;
  const uint64_t* smask;
  const uint8_t* inside;
  float* ga_xy;
  float* gb_xy;
};

// Per-kernel timing of a context (dgal_set_profiling): each launch is
// bracketed by two events on its stream and waited for, and its duration is
// added to its kernel's total.  Names are string literals.
struct Profiler {
  static constexpr int kMax = 48;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int n = 0;
  const char* name[kMax];
  int64_t launches[kMax];
  double ms[kMax];
  hipError_t err = hipSuccess;
};

inline void prof_begin(Profiler* p, hipStream_t s) {
  if (p != nullptr && p->err == hipSuccess) p->err = hipEventRecord(p->e0, s);
}

inline void prof_end(Profiler* p, const char* name, hipStream_t s) {
  if (p == nullptr || p->err != hipSuccess) return;
  float t = 0.f;
  if ((p->err = hipEventRecord(p->e1, s)) != hipSuccess) return;
  if ((p->err = hipEventSynchronize(p->e1)) != hipSuccess) return;
  if ((p->err = hipEventElapsedTime(&t, p->e0, p->e1)) != hipSuccess) return;
  int k = 0;
  while (k < p->n && __builtin_strcmp(p->name[k], name) != 0) ++k;
  if (k == p->n) {
    if (p->n == Profiler::kMax) return;
    p->name[k] = name;
    p->launches[k] = 0;
    p->ms[k] = 0.0;
    ++p->n;
  }
  ++p->launches[k];
  p->ms[k] += t;
}

// What the kernels need from a context.
struct CtxView {
  int device;
  int cus;          // compute units of the device
  int* err;         // sticky device error word
  int64_t* prefix;  // [2][DGAL_MAX_SEGMENTS + 1]: tile and row-group prefixes
  int64_t* scan;    // [kScanTotals]: per-chunk totals of the tile scan
  Profiler* prof;   // per-kernel timing, or NULL
  unsigned long long* stats;  // path statistics: pairs evaluated, fp64 signs, fp64 areas (NULL: off)
};

// Chunks of 4096 tiles the tile scan can combine (2^24 tiles per call).
constexpr int64_t kScanTotals = 4096;

inline bool aligned(const void* p, uintptr_t a) {
  return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0;
}

// Register capacity for polygons of up to kmax vertices.
inline int reg_k(int kmax_a, int kmax_b) { return (kmax_a <= 4 && kmax_b <= 4) ? 4 : 8; }

inline bool valid_polys(const dgal_polys& p) {
  if (p.count < 0 || p.kmax < 3 || p.kmax > 8) return false;
  if (p.count > 0 && (p.xy == nullptr || !aligned(p.xy, 8))) return false;
  if ((p.zlo == nullptr) != (p.zhi == nullptr)) return false;
  return true;
}

inline PolyArgs poly_args(const dgal_polys& p, int K) {
  PolyArgs a;
  a.xy = p.xy;
  a.nv = p.nv;
  a.zlo = p.zlo;
  a.zhi = p.zhi;
  a.count = p.count;
  a.kmax = p.kmax;
  a.vec4 = (p.kmax == K) && aligned(p.xy, 16);
  return a;
}

inline bool same_polys(const dgal_polys& a, const dgal_polys& b) {
  return a.xy == b.xy && a.nv == b.nv && a.zlo == b.zlo && a.zhi == b.zhi && a.count == b.count &&
         a.kmax == b.kmax;
}

// Switches to a device for the duration of a call, restoring the caller's.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int matrix_forward(const CtxView& ctx, dgal_polys a, dgal_polys b, const int64_t* a_off,
                   const int64_t* b_off, const int64_t* out_off, int nseg, int self_pairs,
                   float* iou, int64_t out_size, dgal_saved* saved, hipStream_t stream,
                   const LaunchShape& shape = LaunchShape());
int matrix_backward(const CtxView& ctx, dgal_polys a, dgal_polys b, const int64_t* a_off,
                    const int64_t* b_off, const int64_t* out_off, int nseg, int self_pairs,
                    const float* grad_iou, int64_t out_size, const dgal_saved* saved,
                    float* grad_a_xy, float* grad_b_xy, float* grad_a_z, float* grad_b_z,
                    hipStream_t stream, const LaunchShape& shape = LaunchShape());

// The allocation-free forward: dgal_iou_matrix with its work list, tile state
// and workspace in the library's static device scratch (matrix.hip).
// matrix_scratch_init takes the scratch's device address once per device
// (that device current); the context does it at creation.
int matrix_scratch_init(int device);
int matrix_forward_noalloc(const CtxView& ctx, dgal_polys a, dgal_polys b, const int64_t* a_off,
                           const int64_t* b_off, const int64_t* out_off, int nseg,
                           int self_pairs, float* iou, int64_t out_size, hipStream_t stream,
                           const LaunchShape& shape = LaunchShape());

// Launchers (return a hipError_t from the launch).
hipError_t launch_pairs_fwd(const PairsFwdArgs& args, int K, bool fixed, bool z3, bool save,
                            hipStream_t stream, const LaunchShape& shape = LaunchShape());
hipError_t launch_pairs_bwd(const PairsBwdArgs& args, int K, bool fixed, bool z3,
                            hipStream_t stream, const LaunchShape& shape = LaunchShape());
hipError_t launch_intersect_fwd(const IntersectArgs& args, int K, bool fixed, hipStream_t stream);
hipError_t launch_intersect_bwd(const IntersectBwdArgs& args, int K, bool fixed,
                                hipStream_t stream);
hipError_t launch_area(const PolyArgs& p, const float* grad, float* out, int K, bool fixed,
                       bool backward, hipStream_t stream);
hipError_t launch_boxes_fwd(const BoxesFwdArgs& args, bool z3, bool save, hipStream_t stream);
hipError_t launch_boxes_bwd(const BoxesBwdArgs& args, bool z3, hipStream_t stream);
hipError_t launch_simple_fwd(const SimpleFwdArgs& args, int K, hipStream_t stream);
hipError_t launch_simple_bwd(const SimpleBwdArgs& args, int K, hipStream_t stream);
// Input-contract status per polygon (status may be NULL) and the number of
// invalid ones (n_bad may be NULL; zeroed first, on the stream); the convex
// contract, or the simple-polygon one.
hipError_t launch_validate(const PolyArgs& p, uint8_t* status, int64_t* n_bad, bool simple,
                           hipStream_t stream);

}  // namespace dgal
