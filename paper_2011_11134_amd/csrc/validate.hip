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

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

}  // namespace

hipError_t launch_validate(const PolyArgs& p, uint8_t* status, int64_t* n_bad,
                           hipStream_t stream) {
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(n_bad);
  if (cnt) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, stream, cnt);
  if (p.count > 0) {
    int64_t blocks = (p.count + kValidateBlock - 1) / kValidateBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(kValidateBlock), 0, stream, p,
                       status, cnt);
  }
  return hipGetLastError();
}

}  // namespace dgal
