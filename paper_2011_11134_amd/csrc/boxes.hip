// boxes.hip -- rotated boxes given by their parameters (Sec. IV-A case
// study: 2D boxes (cx, cy, w, l, yaw), 3D boxes with (z, h) appended), with
// the corners formed in-kernel: the IoU forward and the backward down to the
// parameters, without a [N][4][2] vertex array in HBM.
#include "geom.hpp"
#include "internal.hpp"

namespace dgal {

constexpr int kBoxBlock = 256;

// Corner offsets from the centre of box b: R(yaw) (+-l/2, +-w/2), counter-
// clockwise from (+l/2, -w/2) (the length along the heading).
struct BoxFrame {
  float cx, cy, c, s;
  float rx[4], ry[4];
};

__device__ __forceinline__ BoxFrame box_frame(const float* b) {
  BoxFrame f;
  f.cx = b[0];
  f.cy = b[1];
  const float hw = 0.5f * b[2], hl = 0.5f * b[3];
  // hardware sine / cosine (absolute error ~2^-21 on the yaw range of boxes,
  // i.e. corner errors ~1e-6 of the box size, far inside the IoU tolerance)
  __sincosf(b[4], &f.s, &f.c);
  const float sl[4] = {1.f, 1.f, -1.f, -1.f}, sw[4] = {-1.f, 1.f, 1.f, -1.f};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float dx = sl[k] * hl, dy = sw[k] * hw;
    f.rx[k] = f.c * dx - f.s * dy;
    f.ry[k] = f.s * dx + f.c * dy;
  }
  return f;
}

__device__ __forceinline__ void box_corners(const BoxFrame& f, Poly<4>& P) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    P.x[k] = f.cx + f.rx[k];
    P.y[k] = f.cy + f.ry[k];
  }
}

// dL/d(cx, cy, w, l, yaw) from the corners' gradient.
__device__ __forceinline__ void box_param_grad(const BoxFrame& f, const float2 (&g)[4],
                                               float (&gp)[5]) {
  const float sl[4] = {1.f, 1.f, -1.f, -1.f}, sw[4] = {-1.f, 1.f, 1.f, -1.f};
  float gcx = 0.f, gcy = 0.f, gw = 0.f, gl = 0.f, gyaw = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    gcx += g[k].x;
    gcy += g[k].y;
    gw += 0.5f * sw[k] * (f.c * g[k].y - f.s * g[k].x);
    gl += 0.5f * sl[k] * (f.c * g[k].x + f.s * g[k].y);
    gyaw += g[k].y * f.rx[k] - g[k].x * f.ry[k];
  }
  gp[0] = gcx;
  gp[1] = gcy;
  gp[2] = gw;
  gp[3] = gl;
  gp[4] = gyaw;
}

template <bool Z3, bool SAVE>
__global__ __launch_bounds__(kBoxBlock) void k_boxes_fwd(BoxesFwdArgs args) {
  constexpr int CAP = 8;
  __shared__ float2 s_pt[CAP * kBoxBlock];
  __shared__ uint16_t s_cd[CAP * kBoxBlock];
  const int tid = threadIdx.x;
  const int dim = Z3 ? 7 : 5;
  for (int64_t i = (int64_t)blockIdx.x * kBoxBlock + tid; i < args.count;
       i += (int64_t)gridDim.x * kBoxBlock) {
    const float* ba = args.a + i * dim;
    const float* bb = args.b + i * dim;
    const BoxFrame fa = box_frame(ba), fb = box_frame(bb);
    Poly<4> P, Q;
    box_corners(fa, P);
    box_corners(fb, Q);
    PairResult<4> r;
    pair_forward<4, true, kBoxBlock>(P, 4, Q, 4, s_pt + tid, s_cd + tid, r);
    count_path(args.stats, r.exact, r.thin);
    float zl1 = 0.f, zh1 = 0.f, zl2 = 0.f, zh2 = 0.f;
    if (Z3) {
      zl1 = ba[5] - 0.5f * ba[6];
      zh1 = ba[5] + 0.5f * ba[6];
      zl2 = bb[5] - 0.5f * bb[6];
      zh2 = bb[5] + 0.5f * bb[6];
    }
    args.iou[i] = Z3 ? iou_3d(r.inter, r.a1, r.a2, r.m, zl1, zh1, zl2, zh2)
                     : iou_2d(r.inter, r.a1, r.a2, r.m);
    if (r.overflow) atomicOr(args.err, kErrCapacity);
    if (SAVE) {
      args.nx[i] = (uint8_t)r.m;
      *reinterpret_cast<uint2*>(args.xflags + i * CAP) = make_uint2(r.codes[0], r.codes[1]);
    }
    // rare: the areas again in fp64, from the corners formed again, and the
    // IoU written again
    if (r.thin) {
      const int64_t i2 = opaque(i);
      box_corners(box_frame(args.a + i2 * dim), P);
      box_corners(box_frame(args.b + i2 * dim), Q);
      stage_pair<4, kBoxBlock>(s_pt + tid, P, Q);
      float inter, a1, a2;
      thin_areas64<4, true, kBoxBlock>(r.m, r.codes, 4, 4, s_pt + tid, inter, a1, a2);
      args.iou[i] = Z3 ? iou_3d(inter, a1, a2, r.m, zl1, zh1, zl2, zh2)
                       : iou_2d(inter, a1, a2, r.m);
    }
  }
}

template <bool Z3>
__global__ __launch_bounds__(kBoxBlock) void k_boxes_bwd(BoxesBwdArgs args) {
  constexpr int CAP = 8;
  __shared__ float2 s_v[CAP * kBoxBlock];
  __shared__ float2 s_g[CAP * kBoxBlock];
  __shared__ uint2 s_tab[256];
  const int tid = threadIdx.x;
  const int dim = Z3 ? 7 : 5;
  fill_code_table<4, true, kBoxBlock>(s_tab);
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * kBoxBlock + tid; i < args.count;
       i += (int64_t)gridDim.x * kBoxBlock) {
    const float* ba = args.a + i * dim;
    const float* bb = args.b + i * dim;
    const BoxFrame fa = box_frame(ba), fb = box_frame(bb);
    Poly<4> P, Q;
    box_corners(fa, P);
    box_corners(fb, Q);
    const uint2 w = *reinterpret_cast<const uint2*>(args.xflags + i * CAP);
    const uint32_t codes[2] = {w.x, w.y};
    float lo1 = 0.f, hi1 = 0.f, lo2 = 0.f, hi2 = 0.f;
    if (Z3) {
      lo1 = ba[5] - 0.5f * ba[6];
      hi1 = ba[5] + 0.5f * ba[6];
      lo2 = bb[5] - 0.5f * bb[6];
      hi2 = bb[5] + 0.5f * bb[6];
    }
    float2 gP[4], gQ[4], gz1, gz2;
    bool thin;
    const float gi = args.grad[i];
    const int nxi = (int)args.nx[i];
    pair_backward<4, true, Z3, kBoxBlock, true>(P, 4, Q, 4, gi, nxi, codes, lo1, hi1, lo2, hi2,
                                                s_v + tid, s_g + tid, s_tab, gP, gQ, gz1, gz2,
                                                thin);
    if (thin) {  // rare: the gradient again in fp64, from the same fp32 corners
      stage_pair<4, kBoxBlock>(s_v + tid, P, Q);
      pair_backward64<4, true, Z3, kBoxBlock>(4, 4, gi, nxi, codes, lo1, hi1, lo2, hi2,
                                              s_v + tid, s_g + tid, gP, gQ, gz1, gz2);
    }
    float gpa[5], gpb[5];
    box_param_grad(fa, gP, gpa);
    box_param_grad(fb, gQ, gpb);
    float* oa = args.ga + i * dim;
    float* ob = args.gb + i * dim;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      oa[t] = gpa[t];
      ob[t] = gpb[t];
    }
    if (Z3) {  // zlo = z - h/2, zhi = z + h/2
      oa[5] = gz1.x + gz1.y;
      oa[6] = 0.5f * (gz1.y - gz1.x);
      ob[5] = gz2.x + gz2.y;
      ob[6] = 0.5f * (gz2.y - gz2.x);
    }
  }
}

namespace {

int box_grid(int64_t n) {
  int64_t blocks = (n + kBoxBlock - 1) / kBoxBlock;
  const int64_t cap = 1 << 20;
  return (int)(blocks < 1 ? 1 : (blocks > cap ? cap : blocks));
}

}  // namespace

hipError_t launch_boxes_fwd(const BoxesFwdArgs& args, bool z3, bool save, hipStream_t stream) {
  const dim3 g(box_grid(args.count)), b(kBoxBlock);
  if (z3) {
    if (save) hipLaunchKernelGGL((k_boxes_fwd<true, true>), g, b, 0, stream, args);
    else hipLaunchKernelGGL((k_boxes_fwd<true, false>), g, b, 0, stream, args);
  } else {
    if (save) hipLaunchKernelGGL((k_boxes_fwd<false, true>), g, b, 0, stream, args);
    else hipLaunchKernelGGL((k_boxes_fwd<false, false>), g, b, 0, stream, args);
  }
  return hipGetLastError();
}

hipError_t launch_boxes_bwd(const BoxesBwdArgs& args, bool z3, hipStream_t stream) {
  const dim3 g(box_grid(args.count)), b(kBoxBlock);
  if (z3) hipLaunchKernelGGL((k_boxes_bwd<true>), g, b, 0, stream, args);
  else hipLaunchKernelGGL((k_boxes_bwd<false>), g, b, 0, stream, args);
  return hipGetLastError();
}

}  // namespace dgal
