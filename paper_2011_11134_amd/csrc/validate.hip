// validate.hip -- the input contract of Sec. III (convex polygons, vertices
// counter-clockwise, at most kmax of them) checked per polygon on the device.
// One lane per polygon, grid-stride.
#include "geom.hpp"
#include "internal.hpp"

namespace dgal {

namespace {

constexpr int kValidateBlock = 256;

// Half-plane of a direction (dx, dy): 0 for angles in [0, pi), 1 for
// [pi, 2 pi).  From the signs of the coordinate differences alone, which are
// the comparisons of the fp32 inputs and hence exact.
__device__ __forceinline__ int half_of(float ax, float ay, float bx, float by) {
  return (by > ay || (by == ay && bx > ax)) ? 0 : 1;
}

// 0 valid; 1 vertex count outside [3, kmax]; 2 a turn that is not strictly
// left (orientation of three consecutive vertices in fp64, as orient64
// evaluates it); 3 every turn left but the boundary winds more than once.
// With every turn left, each edge direction turns by less than half a turn
// from the previous one, so the direction passes angle 0 exactly when it goes
// from the lower half-plane to the upper one; the number of such steps is
// the winding number.
__device__ int polygon_status(const float* __restrict__ xy, int n, int kmax) {
  if (n < 3 || n > kmax) return 1;
  float x[8], y[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float2 v = k < n ? reinterpret_cast<const float2*>(xy)[k] : make_float2(0.f, 0.f);
    x[k] = v.x;
    y[k] = v.y;
  }
  int wraps = 0;
  bool left = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < n) {
      const int kp = k == 0 ? n - 1 : k - 1, kn = k + 1 < n ? k + 1 : 0;
      // dynamic neighbours through selects over the static slots
      float px = x[0], py = y[0], nxv = x[0], nyv = y[0];
#pragma unroll
      for (int t = 1; t < 8; ++t) {
        px = t == kp ? x[t] : px;
        py = t == kp ? y[t] : py;
        nxv = t == kn ? x[t] : nxv;
        nyv = t == kn ? y[t] : nyv;
      }
      left = left && orient64(px, py, x[k], y[k], nxv, nyv) > 0.0;
      wraps += (half_of(px, py, x[k], y[k]) == 1 && half_of(x[k], y[k], nxv, nyv) == 0) ? 1 : 0;
    }
  }
  if (!left) return 2;
  return wraps == 1 ? 0 : 3;
}

__global__ __launch_bounds__(kValidateBlock) void k_validate(PolyArgs p, uint8_t* status,
                                                             unsigned long long* n_bad) {
  unsigned long long bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * kValidateBlock + threadIdx.x; i < p.count;
       i += (int64_t)gridDim.x * kValidateBlock) {
    const int n = p.nv ? (int)p.nv[i] : p.kmax;
    const int st = polygon_status(p.xy + i * (int64_t)p.kmax * 2, n, p.kmax);
    if (status) status[i] = (uint8_t)st;
    bad += st != 0;
  }
  // one global atomic per wavefront
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
  if (n_bad && (threadIdx.x & 63) == 0 && bad) atomicAdd(n_bad, bad);
}

// Simple-polygon contract (the extension of Sec. III to arbitrary shapes):
// 0 valid; 1 vertex count outside [3, kmax]; 2 two non-adjacent edges touch
// or cross, or two adjacent edges fold back onto each other; 3 shoelace area
// not positive (clockwise or flat).  Every test is an fp64 sign of the fp32
// vertices evaluated in a fixed order without contraction.
__device__ int simple_status(const float* __restrict__ xy, int n, int kmax) {
#pragma clang fp contract(off)
  if (n < 3 || n > kmax) return 1;
  float x[8], y[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float2 v = k < n ? reinterpret_cast<const float2*>(xy)[k] : make_float2(0.f, 0.f);
    x[k] = v.x;
    y[k] = v.y;
  }
  auto sgn = [](double v) { return (v > 0.0) - (v < 0.0); };
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
#pragma unroll
    for (int j = i + 1; j < 8; ++j) {
      if (j < n && ok) {
        const int i1 = i + 1 < n ? i + 1 : 0, j1 = j + 1 < n ? j + 1 : 0;
        // dynamic ends through selects over the static slots
        float bx = x[0], by = y[0], dx = x[0], dy = y[0];
#pragma unroll
        for (int t = 1; t < 8; ++t) {
          bx = t == i1 ? x[t] : bx;
          by = t == i1 ? y[t] : by;
          dx = t == j1 ? x[t] : dx;
          dy = t == j1 ? y[t] : dy;
        }
        const float ax = x[i], ay = y[i], cx = x[j], cy = y[j];
        const bool adjacent = (j == i + 1) || (i == 0 && j == n - 1);
        if (adjacent) {
          // shared vertex s, far ends u (edge i) and w (edge j)
          const bool first = j == i + 1;
          const float sx = first ? bx : ax, sy = first ? by : ay;
          const float ux = first ? ax : bx, uy = first ? ay : by;
          const float wx = first ? dx : cx, wy = first ? dy : cy;
          const double dot = ((double)ux - (double)sx) * ((double)wx - (double)sx) +
                             ((double)uy - (double)sy) * ((double)wy - (double)sy);
          if (orient64(ux, uy, sx, sy, wx, wy) == 0.0 && dot > 0.0) ok = false;
        } else {
          const int s1 = sgn(orient64(cx, cy, dx, dy, ax, ay));
          const int s2 = sgn(orient64(cx, cy, dx, dy, bx, by));
          const int s3 = sgn(orient64(ax, ay, bx, by, cx, cy));
          const int s4 = sgn(orient64(ax, ay, bx, by, dx, dy));
          if (s1 * s2 <= 0 && s3 * s4 <= 0) {
            bool apart = false;
            if (s1 == 0 && s2 == 0 && s3 == 0 && s4 == 0) {
              apart = fmaxf(ax, bx) < fminf(cx, dx) || fmaxf(cx, dx) < fminf(ax, bx) ||
                      fmaxf(ay, by) < fminf(cy, dy) || fmaxf(cy, dy) < fminf(ay, by);
            }
            if (!apart) ok = false;
          }
        }
      }
    }
  }
  if (!ok) return 2;
  double area = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < n) {
      const int k1 = k + 1 < n ? k + 1 : 0;
      float nx = x[0], ny = y[0];
#pragma unroll
      for (int t = 1; t < 8; ++t) {
        nx = t == k1 ? x[t] : nx;
        ny = t == k1 ? y[t] : ny;
      }
      area += (double)x[k] * (double)ny - (double)nx * (double)y[k];
    }
  }
  return 0.5 * area > 0.0 ? 0 : 3;
}

__global__ __launch_bounds__(kValidateBlock) void k_validate_simple(PolyArgs p, uint8_t* status,
                                                                    unsigned long long* n_bad) {
  unsigned long long bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * kValidateBlock + threadIdx.x; i < p.count;
       i += (int64_t)gridDim.x * kValidateBlock) {
    const int n = p.nv ? (int)p.nv[i] : p.kmax;
    const int st = simple_status(p.xy + i * (int64_t)p.kmax * 2, n, p.kmax);
    if (status) status[i] = (uint8_t)st;
    bad += st != 0;
  }
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
  if (n_bad && (threadIdx.x & 63) == 0 && bad) atomicAdd(n_bad, bad);
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

}  // namespace

hipError_t launch_validate(const PolyArgs& p, uint8_t* status, int64_t* n_bad, bool simple,
                           hipStream_t stream) {
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(n_bad);
  if (cnt) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, stream, cnt);
  if (p.count > 0) {
    int64_t blocks = (p.count + kValidateBlock - 1) / kValidateBlock;
    if (blocks > 65536) blocks = 65536;
    if (simple)
      hipLaunchKernelGGL(k_validate_simple, dim3((unsigned)blocks), dim3(kValidateBlock), 0,
                         stream, p, status, cnt);
    else
      hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(kValidateBlock), 0, stream, p,
                         status, cnt);
  }
  return hipGetLastError();
}

}  // namespace dgal
