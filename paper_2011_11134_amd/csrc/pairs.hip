// pairs.hip -- elementwise-pair IoU forward and backward kernels (Sec. II-B
// listing, batched): one wavefront lane per polygon pair, grid-stride.
#include <type_traits>

#include "geom.hpp"
#include "internal.hpp"

namespace dgal {

template <int K>
constexpr int pairs_block() {
  return K == 8 ? 128 : 256;
}

template <int K, bool FIXED, bool Z3, bool SAVE>
__global__ __launch_bounds__(pairs_block<K>())
__attribute__((amdgpu_waves_per_eu(fwd_waves_per_simd<K>()))) void k_pairs_fwd(PairsFwdArgs args) {
  constexpr int BLOCK = pairs_block<K>();
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
    pair_forward<K, FIXED, BLOCK>(P, n1, Q, n2, s_pt + tid, s_cd + tid, r);
    count_path(args.stats, r.exact, r.thin);
    args.iou[i] = pair_iou<Z3>(r.inter, r.a1, r.a2, r.m, args.a.zlo, args.a.zhi, i, args.b.zlo,
                               args.b.zhi, i);
    if (r.overflow) atomicOr(args.err, kErrCapacity);
    if (SAVE) {
      args.nx[i] = (uint8_t)r.m;
      uint8_t* row = args.xflags + i * (int64_t)args.cap;
      if (FIXED || args.flags_vec) {
        if constexpr (K == 4) {
          *reinterpret_cast<uint2*>(row) = make_uint2(r.codes[0], r.codes[1]);
        } else {
          *reinterpret_cast<uint4*>(row) = make_uint4(r.codes[0], r.codes[1], r.codes[2], r.codes[3]);
        }
      } else {
#pragma unroll
        for (int k = 0; k < CAP; ++k) {
          if (k < args.cap) row[k] = (uint8_t)(r.codes[k >> 2] >> ((k & 3) * 8));
        }
      }
    }
    // rare: the areas again in fp64, from the polygons reloaded, and the IoU
    // written again (last, so that nothing of it is live on the common path)
    if (r.thin) {
      const int64_t i2 = opaque(i);
      load_poly<K, FIXED>(args.a.xy, i2, args.a.kmax, args.a.vec4, n1, P);
      load_poly<K, FIXED>(args.b.xy, i2, args.b.kmax, args.b.vec4, n2, Q);
      stage_pair<K, BLOCK>(s_pt + tid, P, Q);
      float inter, a1, a2;
      thin_areas64<K, FIXED, BLOCK>(r.m, r.codes, n1, n2, s_pt + tid, inter, a1, a2);
      args.iou[i] = pair_iou<Z3>(inter, a1, a2, r.m, args.a.zlo, args.a.zhi, i, args.b.zlo,
                                 args.b.zhi, i);
    }
  }
}

template <int K, bool FIXED, bool Z3>
__global__ __launch_bounds__(pairs_block<K>()) void k_pairs_bwd(PairsBwdArgs args) {
  constexpr int BLOCK = pairs_block<K>();
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
    uint32_t codes[K / 2];
    const uint8_t* row = args.xflags + i * (int64_t)args.cap;
    if (FIXED || args.flags_vec) {
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
        if (k < args.cap) {
          const uint32_t c = row[k];
          codes[k >> 2] = (codes[k >> 2] & ~(0xffu << ((k & 3) * 8))) | (c << ((k & 3) * 8));
        }
      }
    }
    float lo1 = 0.f, hi1 = 0.f, lo2 = 0.f, hi2 = 0.f;
    if (Z3) {
      lo1 = args.a.zlo[i];
      hi1 = args.a.zhi[i];
      lo2 = args.b.zlo[i];
      hi2 = args.b.zhi[i];
    }
    float2 gP[K], gQ[K], gz1, gz2;
    bool thin;
    const float gi = args.grad[i];
    const int nxi = (int)args.nx[i];
    pair_backward<K, FIXED, Z3, BLOCK, true>(P, n1, Q, n2, gi, nxi, codes, lo1, hi1, lo2, hi2,
                                             s_v + tid, s_g + tid, s_tab, gP, gQ, gz1, gz2, thin);
    if (thin) {  // rare: the gradient again in fp64, from the polygons reloaded
      const int64_t i2 = opaque(i);
      load_poly<K, FIXED>(args.a.xy, i2, args.a.kmax, args.a.vec4, n1, P);
      load_poly<K, FIXED>(args.b.xy, i2, args.b.kmax, args.b.vec4, n2, Q);
      stage_pair<K, BLOCK>(s_v + tid, P, Q);
      pair_backward64<K, FIXED, Z3, BLOCK>(n1, n2, gi, nxi, codes, lo1, hi1, lo2, hi2, s_v + tid,
                                           s_g + tid, gP, gQ, gz1, gz2);
    }
    float* oa = args.ga_xy + i * (int64_t)args.a.kmax * 2;
    float* ob = args.gb_xy + i * (int64_t)args.b.kmax * 2;
    if (FIXED || args.a.vec4) {
#pragma unroll
      for (int k = 0; k < K; k += 2)
        *reinterpret_cast<float4*>(oa + 2 * k) = make_float4(gP[k].x, gP[k].y, gP[k + 1].x, gP[k + 1].y);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < args.a.kmax) *reinterpret_cast<float2*>(oa + 2 * k) = gP[k];
    }
    if (FIXED || args.b.vec4) {
#pragma unroll
      for (int k = 0; k < K; k += 2)
        *reinterpret_cast<float4*>(ob + 2 * k) = make_float4(gQ[k].x, gQ[k].y, gQ[k + 1].x, gQ[k + 1].y);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < args.b.kmax) *reinterpret_cast<float2*>(ob + 2 * k) = gQ[k];
    }
    if (Z3) {
      *reinterpret_cast<float2*>(args.ga_z + 2 * i) = gz1;
      *reinterpret_cast<float2*>(args.gb_z + 2 * i) = gz2;
    }
  }
}

namespace {

int grid_for(int64_t n, int block, int64_t want = 0) {
  int64_t blocks = (n + block - 1) / block;
  if (want > 0 && want < blocks) blocks = want;  // persistent grid-stride launch
  const int64_t cap = 1 << 20;  // grid-stride beyond this
  return (int)(blocks < 1 ? 1 : (blocks > cap ? cap : blocks));
}

template <int K, bool FIXED, bool Z3>
hipError_t fwd3(const PairsFwdArgs& a, bool save, hipStream_t s, int64_t g) {
  constexpr int B = pairs_block<K>();
  const dim3 grid(grid_for(a.a.count, B, g));
  if (save)
    hipLaunchKernelGGL((k_pairs_fwd<K, FIXED, Z3, true>), grid, dim3(B), 0, s, a);
  else
    hipLaunchKernelGGL((k_pairs_fwd<K, FIXED, Z3, false>), grid, dim3(B), 0, s, a);
  return hipGetLastError();
}

template <int K, bool FIXED>
hipError_t fwd2(const PairsFwdArgs& a, bool z3, bool save, hipStream_t s, int64_t g) {
  return z3 ? fwd3<K, FIXED, true>(a, save, s, g) : fwd3<K, FIXED, false>(a, save, s, g);
}

template <int K, bool FIXED, bool Z3>
hipError_t bwd3(const PairsBwdArgs& a, hipStream_t s, int64_t g) {
  constexpr int B = pairs_block<K>();
  hipLaunchKernelGGL((k_pairs_bwd<K, FIXED, Z3>), dim3(grid_for(a.a.count, B, g)), dim3(B), 0, s,
                     a);
  return hipGetLastError();
}

template <int K, bool FIXED>
hipError_t bwd2(const PairsBwdArgs& a, bool z3, hipStream_t s, int64_t g) {
  return z3 ? bwd3<K, FIXED, true>(a, s, g) : bwd3<K, FIXED, false>(a, s, g);
}

}  // namespace

hipError_t launch_pairs_fwd(const PairsFwdArgs& args, int K, bool fixed, bool z3, bool save,
                            hipStream_t stream, const LaunchShape& shape) {
  const int64_t g = shape.grid;
  if (K == 4)
    return fixed ? fwd2<4, true>(args, z3, save, stream, g) : fwd2<4, false>(args, z3, save, stream, g);
  return fixed ? fwd2<8, true>(args, z3, save, stream, g) : fwd2<8, false>(args, z3, save, stream, g);
}

hipError_t launch_pairs_bwd(const PairsBwdArgs& args, int K, bool fixed, bool z3,
                            hipStream_t stream, const LaunchShape& shape) {
  const int64_t g = shape.grid;
  if (K == 4) return fixed ? bwd2<4, true>(args, z3, stream, g) : bwd2<4, false>(args, z3, stream, g);
  return fixed ? bwd2<8, true>(args, z3, stream, g) : bwd2<8, false>(args, z3, stream, g);
}

}  // namespace dgal
