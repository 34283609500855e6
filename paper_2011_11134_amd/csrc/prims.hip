// prims.hip -- the geometry primitives under the IoU, exported on their own
// (Sec. II-B: the intersection of two convex polygons with its vertex count
// and provenance flags; Sec. III: polygon area), each with its backward.  One
// wavefront lane per pair / polygon, grid-stride.
#include "geom.hpp"
#include "internal.hpp"

namespace dgal {

template <int K>
constexpr int prim_block() {
  return K == 8 ? 128 : 256;
}

// Intersection polygon of each pair: ordered vertices (absolute frame, cap
// slots per row, 0 past nx), nx and xflags.
template <int K, bool FIXED>
__global__ __launch_bounds__(prim_block<K>())
__attribute__((amdgpu_waves_per_eu(fwd_waves_per_simd<K>()))) void k_intersect_fwd(IntersectArgs args) {
  constexpr int BLOCK = prim_block<K>();
  constexpr int CAP = 2 * K;
  __shared__ float2 s_pt[CAP * BLOCK];
  __shared__ uint16_t s_cd[CAP * BLOCK];
  const int tid = threadIdx.x;
  const int64_t n = args.a.count;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + tid; i < n; i += (int64_t)gridDim.x * BLOCK) {
    const int n1 = FIXED ? K : poly_count(args.a.nv, i, args.a.kmax);
    const int n2 = FIXED ? K : poly_count(args.b.nv, i, args.b.kmax);
    Poly<K> P, Q;
    load_poly<K, FIXED>(args.a.xy, i, args.a.kmax, args.a.vec4, n1, P);
    load_poly<K, FIXED>(args.b.xy, i, args.b.kmax, args.b.vec4, n2, Q);
    PairResult<K> r;
    float2 ov[CAP];
    pair_forward<K, FIXED, BLOCK, true>(P, n1, Q, n2, s_pt + tid, s_cd + tid, r, ov);
    count_path(args.stats, r.exact, false);  // vertices only: no areas to rebuild
    if (r.overflow) atomicOr(args.err, kErrCapacity);
    args.nx[i] = (uint8_t)r.m;
    uint8_t* row = args.xflags + i * (int64_t)args.cap;
    float2* out = reinterpret_cast<float2*>(args.out_xy) + i * (int64_t)args.cap;
    if (FIXED || args.rows_vec) {  // cap == 2K, rows 16-byte aligned
#pragma unroll
      for (int k = 0; k < CAP; k += 2)
        *reinterpret_cast<float4*>(out + k) = make_float4(ov[k].x, ov[k].y, ov[k + 1].x, ov[k + 1].y);
      if constexpr (K == 4) {
        *reinterpret_cast<uint2*>(row) = make_uint2(r.codes[0], r.codes[1]);
      } else {
        *reinterpret_cast<uint4*>(row) = make_uint4(r.codes[0], r.codes[1], r.codes[2], r.codes[3]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < CAP; ++k) {
        if (k < args.cap) {
          out[k] = ov[k];
          row[k] = (uint8_t)(r.codes[k >> 2] >> ((k & 3) * 8));
        }
      }
    }
  }
}

// Gradient of sum <grad_xy, X> over the saved intersection vertices.
template <int K, bool FIXED>
__global__ __launch_bounds__(prim_block<K>()) void k_intersect_bwd(IntersectBwdArgs args) {
  constexpr int BLOCK = prim_block<K>();
  constexpr int CAP = 2 * K;
  __shared__ float2 s_v[CAP * BLOCK];
  __shared__ float2 s_g[CAP * BLOCK];
  __shared__ uint2 s_tab[256];
  const int tid = threadIdx.x;
  fill_code_table<K, FIXED, BLOCK>(s_tab);
  __syncthreads();
  const int64_t n = args.a.count;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + tid; i < n; i += (int64_t)gridDim.x * BLOCK) {
    const int n1 = FIXED ? K : poly_count(args.a.nv, i, args.a.kmax);
    const int n2 = FIXED ? K : poly_count(args.b.nv, i, args.b.kmax);
    Poly<K> P, Q;
    load_poly<K, FIXED>(args.a.xy, i, args.a.kmax, args.a.vec4, n1, P);
    load_poly<K, FIXED>(args.b.xy, i, args.b.kmax, args.b.vec4, n2, Q);
    const uint8_t* row = args.xflags + i * (int64_t)args.cap;
    const float2* gin = reinterpret_cast<const float2*>(args.grad_xy) + i * (int64_t)args.cap;
    uint32_t codes[K / 2];
    float2 G[CAP];
    if (FIXED || args.rows_vec) {  // whole rows in 16-byte (8-byte flag) loads
      if constexpr (K == 4) {
        const uint2 c = *reinterpret_cast<const uint2*>(row);
        codes[0] = c.x;
        codes[1] = c.y;
      } else {
        const uint4 c = *reinterpret_cast<const uint4*>(row);
        codes[0] = c.x;
        codes[1] = c.y;
        codes[2] = c.z;
        codes[3] = c.w;
      }
#pragma unroll
      for (int k = 0; k < CAP; k += 2) {
        const float4 v = *reinterpret_cast<const float4*>(gin + k);
        G[k] = make_float2(v.x, v.y);
        G[k + 1] = make_float2(v.z, v.w);
      }
    } else {
#pragma unroll
      for (int w = 0; w < K / 2; ++w) codes[w] = 0xffffffffu;
#pragma unroll
      for (int k = 0; k < CAP; ++k) {
        if (k < args.cap) {
          const uint32_t c = row[k];
          codes[k >> 2] = (codes[k >> 2] & ~(0xffu << ((k & 3) * 8))) | (c << ((k & 3) * 8));
          G[k] = gin[k];
        } else {
          G[k] = make_float2(0.f, 0.f);
        }
      }
    }
    float2 gP[K], gQ[K];
    pair_vertex_backward<K, FIXED, BLOCK>(P, n1, Q, n2, (int)args.nx[i], codes, G, s_v + tid,
                                          s_g + tid, s_tab, gP, gQ);
    float* oa = args.ga_xy + i * (int64_t)args.a.kmax * 2;
    float* ob = args.gb_xy + i * (int64_t)args.b.kmax * 2;
    if (FIXED) {  // rows of exactly K vertices, 16-byte aligned
#pragma unroll
      for (int k = 0; k < K; k += 2) {
        *reinterpret_cast<float4*>(oa + 2 * k) = make_float4(gP[k].x, gP[k].y, gP[k + 1].x, gP[k + 1].y);
        *reinterpret_cast<float4*>(ob + 2 * k) = make_float4(gQ[k].x, gQ[k].y, gQ[k + 1].x, gQ[k + 1].y);
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k < args.a.kmax) *reinterpret_cast<float2*>(oa + 2 * k) = gP[k];
        if (k < args.b.kmax) *reinterpret_cast<float2*>(ob + 2 * k) = gQ[k];
      }
    }
  }
}

// Area of each polygon, and the gradient of sum g * area.
template <int K, bool FIXED>
__global__ __launch_bounds__(256) void k_area_fwd(PolyArgs p, float* area) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < p.count;
       i += (int64_t)gridDim.x * 256) {
    const int n = FIXED ? K : poly_count(p.nv, i, p.kmax);
    Poly<K> P;
    load_poly<K, FIXED>(p.xy, i, p.kmax, p.vec4, n, P);
    area[i] = poly_area<K, FIXED>(P, n);
  }
}

template <int K, bool FIXED>
__global__ __launch_bounds__(256) void k_area_bwd(PolyArgs p, const float* grad, float* gxy) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < p.count;
       i += (int64_t)gridDim.x * 256) {
    const int n = FIXED ? K : poly_count(p.nv, i, p.kmax);
    Poly<K> P;
    load_poly<K, FIXED>(p.xy, i, p.kmax, p.vec4, n, P);
    float2 gv[K];
    poly_area_grad<K, FIXED>(P, n, grad[i], gv);
    float* o = gxy + i * (int64_t)p.kmax * 2;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < p.kmax) *reinterpret_cast<float2*>(o + 2 * k) = gv[k];
  }
}

namespace {

int grid_of(int64_t n, int block) {
  int64_t blocks = (n + block - 1) / block;
  const int64_t cap = 1 << 20;
  return (int)(blocks < 1 ? 1 : (blocks > cap ? cap : blocks));
}

template <int K>
hipError_t isect_fwd(const IntersectArgs& a, bool fixed, hipStream_t s) {
  constexpr int B = prim_block<K>();
  if (fixed)
    hipLaunchKernelGGL((k_intersect_fwd<K, true>), dim3(grid_of(a.a.count, B)), dim3(B), 0, s, a);
  else
    hipLaunchKernelGGL((k_intersect_fwd<K, false>), dim3(grid_of(a.a.count, B)), dim3(B), 0, s, a);
  return hipGetLastError();
}

template <int K>
hipError_t isect_bwd(const IntersectBwdArgs& a, bool fixed, hipStream_t s) {
  constexpr int B = prim_block<K>();
  if (fixed)
    hipLaunchKernelGGL((k_intersect_bwd<K, true>), dim3(grid_of(a.a.count, B)), dim3(B), 0, s, a);
  else
    hipLaunchKernelGGL((k_intersect_bwd<K, false>), dim3(grid_of(a.a.count, B)), dim3(B), 0, s, a);
  return hipGetLastError();
}

template <int K>
hipError_t area_launch(const PolyArgs& p, const float* grad, float* out, bool fixed, bool bwd,
                       hipStream_t s) {
  const dim3 g(grid_of(p.count, 256)), b(256);
  if (bwd) {
    if (fixed) hipLaunchKernelGGL((k_area_bwd<K, true>), g, b, 0, s, p, grad, out);
    else hipLaunchKernelGGL((k_area_bwd<K, false>), g, b, 0, s, p, grad, out);
  } else {
    if (fixed) hipLaunchKernelGGL((k_area_fwd<K, true>), g, b, 0, s, p, out);
    else hipLaunchKernelGGL((k_area_fwd<K, false>), g, b, 0, s, p, out);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_intersect_fwd(const IntersectArgs& args, int K, bool fixed, hipStream_t stream) {
  return K == 4 ? isect_fwd<4>(args, fixed, stream) : isect_fwd<8>(args, fixed, stream);
}

hipError_t launch_intersect_bwd(const IntersectBwdArgs& args, int K, bool fixed,
                                hipStream_t stream) {
  return K == 4 ? isect_bwd<4>(args, fixed, stream) : isect_bwd<8>(args, fixed, stream);
}

hipError_t launch_area(const PolyArgs& p, const float* grad, float* out, int K, bool fixed,
                       bool backward, hipStream_t stream) {
  return K == 4 ? area_launch<4>(p, grad, out, fixed, backward, stream)
                : area_launch<8>(p, grad, out, fixed, backward, stream);
}

}  // namespace dgal
