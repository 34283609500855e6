// api.hip -- the C ABI declared in include/dgal.h: argument validation on the
// host, then kernel dispatch on the caller's stream.  No allocation per call.
#include <new>

#include "internal.hpp"

struct dgal_ctx {
  dgal::CtxView v;
};

namespace {

using dgal::aligned;
using dgal::DeviceGuard;
using dgal::poly_args;
using dgal::reg_k;
using dgal::valid_polys;

int status_of(hipError_t e) { return e == hipSuccess ? DGAL_OK : DGAL_EHIP; }

}  // namespace

extern "C" {

int dgal_create(dgal_ctx** out, int hip_device) {
  if (out == nullptr) return DGAL_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return DGAL_EHIP;
  if (hip_device < 0 || hip_device >= ndev) return DGAL_EINVAL;
  DeviceGuard g(hip_device);
  if (!g.ok) return DGAL_EHIP;
  dgal_ctx* c = new (std::nothrow) dgal_ctx;
  if (c == nullptr) return DGAL_EHIP;
  c->v.device = hip_device;
  c->v.err = nullptr;
  c->v.prefix = nullptr;
  c->v.scan = nullptr;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess ||
      cus <= 0)
    cus = 256;
  c->v.cus = cus;
  if (hipMalloc(reinterpret_cast<void**>(&c->v.err), sizeof(int)) != hipSuccess ||
      hipMemset(c->v.err, 0, sizeof(int)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&c->v.prefix), sizeof(int64_t) * 2 * (DGAL_MAX_SEGMENTS + 1)) !=
          hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&c->v.scan), sizeof(int64_t) * dgal::kScanTotals) !=
          hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    if (c->v.err) (void)hipFree(c->v.err);
    if (c->v.prefix) (void)hipFree(c->v.prefix);
    if (c->v.scan) (void)hipFree(c->v.scan);
    delete c;
    return DGAL_EHIP;
  }
  *out = c;
  return DGAL_OK;
}

void dgal_destroy(dgal_ctx* ctx) {
  if (ctx == nullptr) return;
  DeviceGuard g(ctx->v.device);
  if (ctx->v.err) (void)hipFree(ctx->v.err);
  if (ctx->v.prefix) (void)hipFree(ctx->v.prefix);
  if (ctx->v.scan) (void)hipFree(ctx->v.scan);
  delete ctx;
}

const char* dgal_status_string(int status) {
  switch (status) {
    case DGAL_OK: return "DGAL_OK";
    case DGAL_EINVAL: return "DGAL_EINVAL: invalid argument";
    case DGAL_ECAPACITY: return "DGAL_ECAPACITY: capacity exceeded";
    case DGAL_EHIP: return "DGAL_EHIP: HIP runtime error";
    default: return "unknown dgal status";
  }
}

int dgal_check(dgal_ctx* ctx, void* stream) {
  if (ctx == nullptr) return DGAL_EINVAL;
  DeviceGuard g(ctx->v.device);
  if (!g.ok) return DGAL_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return DGAL_EHIP;
  int host = 0;
  if (hipMemcpy(&host, ctx->v.err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return DGAL_EHIP;
  if (host != 0) {
    if (hipMemset(ctx->v.err, 0, sizeof(int)) != hipSuccess) return DGAL_EHIP;
    if (host & dgal::kErrCapacity) return DGAL_ECAPACITY;
    return DGAL_EINVAL;
  }
  return DGAL_OK;
}

int dgal_iou_pairs(dgal_ctx* ctx, dgal_polys a, dgal_polys b, float* iou, uint8_t* nx,
                   uint8_t* xflags, void* stream) {
  if (ctx == nullptr || !valid_polys(a) || !valid_polys(b)) return DGAL_EINVAL;
  if (a.count != b.count) return DGAL_EINVAL;
  if ((nx == nullptr) != (xflags == nullptr)) return DGAL_EINVAL;
  if ((a.zlo == nullptr) != (b.zlo == nullptr)) return DGAL_EINVAL;
  if (a.count > 0 && iou == nullptr) return DGAL_EINVAL;
  if (a.count == 0) return DGAL_OK;
  DeviceGuard g(ctx->v.device);
  if (!g.ok) return DGAL_EHIP;
  const int K = reg_k(a.kmax, b.kmax);
  dgal::PairsFwdArgs args;
  args.a = poly_args(a, K);
  args.b = poly_args(b, K);
  args.iou = iou;
  args.nx = nx;
  args.xflags = xflags;
  args.cap = a.kmax + b.kmax;
  args.flags_vec = args.cap == 2 * K && aligned(xflags, (uintptr_t)(2 * K));
  args.err = ctx->v.err;
  // the fixed-size kernels also assume vector-aligned rows of coordinates and codes
  const bool fixed = a.nv == nullptr && b.nv == nullptr && a.kmax == K && b.kmax == K &&
                     args.a.vec4 && args.b.vec4 && (nx == nullptr || args.flags_vec);
  return status_of(dgal::launch_pairs_fwd(args, K, fixed, a.zlo != nullptr, nx != nullptr,
                                          static_cast<hipStream_t>(stream)));
}

int dgal_iou_backward(dgal_ctx* ctx, int32_t mode, dgal_polys a, dgal_polys b,
                      const int64_t* a_off, const int64_t* b_off, const int64_t* out_off,
                      int32_t nseg, int32_t self_pairs, const float* grad_iou, int64_t out_size,
                      const uint8_t* nx, const uint8_t* xflags, const dgal_saved* saved,
                      float* grad_a_xy, float* grad_b_xy, float* grad_a_z, float* grad_b_z,
                      void* stream) {
  if (ctx == nullptr || !valid_polys(a) || !valid_polys(b)) return DGAL_EINVAL;
  const bool z3 = a.zlo != nullptr;
  if ((a.zlo == nullptr) != (b.zlo == nullptr)) return DGAL_EINVAL;
  if (mode == DGAL_PAIRS) {
    (void)a_off;
    (void)b_off;
    (void)out_off;
    (void)nseg;
    (void)self_pairs;
    (void)saved;
    (void)out_size;
    if (a.count != b.count) return DGAL_EINVAL;
    if (a.count == 0) return DGAL_OK;
    if (grad_iou == nullptr || nx == nullptr || xflags == nullptr || grad_a_xy == nullptr ||
        grad_b_xy == nullptr)
      return DGAL_EINVAL;
    if (z3 != (grad_a_z != nullptr) || z3 != (grad_b_z != nullptr)) return DGAL_EINVAL;
    if (!aligned(grad_a_xy, 8) || !aligned(grad_b_xy, 8)) return DGAL_EINVAL;
    if (z3 && (!aligned(grad_a_z, 8) || !aligned(grad_b_z, 8))) return DGAL_EINVAL;
    DeviceGuard g(ctx->v.device);
    if (!g.ok) return DGAL_EHIP;
    const int K = reg_k(a.kmax, b.kmax);
    dgal::PairsBwdArgs args;
    args.a = poly_args(a, K);
    args.b = poly_args(b, K);
    // the gradient rows are written with the same vector width as the inputs
    args.a.vec4 = args.a.vec4 && aligned(grad_a_xy, 16);
    args.b.vec4 = args.b.vec4 && aligned(grad_b_xy, 16);
    args.grad = grad_iou;
    args.nx = nx;
    args.xflags = xflags;
    args.cap = a.kmax + b.kmax;
    args.flags_vec = args.cap == 2 * K && aligned(xflags, (uintptr_t)(2 * K));
    args.ga_xy = grad_a_xy;
    args.gb_xy = grad_b_xy;
    args.ga_z = grad_a_z;
    args.gb_z = grad_b_z;
    const bool fixed = a.nv == nullptr && b.nv == nullptr && a.kmax == K && b.kmax == K &&
                       args.a.vec4 && args.b.vec4 && args.flags_vec;
    return status_of(dgal::launch_pairs_bwd(args, K, fixed, z3, static_cast<hipStream_t>(stream)));
  }
  if (mode == DGAL_MATRIX) {
    return dgal::matrix_backward(ctx->v, a, b, a_off, b_off, out_off, nseg,
                                 self_pairs, grad_iou, out_size, saved, grad_a_xy, grad_b_xy,
                                 grad_a_z, grad_b_z, static_cast<hipStream_t>(stream));
  }
  return DGAL_EINVAL;
}

int dgal_iou_matrix(dgal_ctx* ctx, dgal_polys a, dgal_polys b, const int64_t* a_off,
                    const int64_t* b_off, const int64_t* out_off, int32_t nseg,
                    int32_t self_pairs, float* iou, int64_t out_size, const dgal_saved* saved,
                    void* stream) {
  if (ctx == nullptr) return DGAL_EINVAL;
  return dgal::matrix_forward(ctx->v, a, b, a_off, b_off, out_off, nseg, self_pairs,
                              iou, out_size, saved, static_cast<hipStream_t>(stream));
}

int dgal_intersect(dgal_ctx* ctx, dgal_polys a, dgal_polys b, float* out_xy, uint8_t* nx,
                   uint8_t* xflags, void* stream) {
  if (ctx == nullptr || !valid_polys(a) || !valid_polys(b)) return DGAL_EINVAL;
  if (a.count != b.count) return DGAL_EINVAL;
  if (a.count == 0) return DGAL_OK;
  if (out_xy == nullptr || nx == nullptr || xflags == nullptr || !aligned(out_xy, 8))
    return DGAL_EINVAL;
  DeviceGuard g(ctx->v.device);
  if (!g.ok) return DGAL_EHIP;
  const int K = reg_k(a.kmax, b.kmax);
  dgal::IntersectArgs args;
  args.a = poly_args(a, K);
  args.b = poly_args(b, K);
  args.out_xy = out_xy;
  args.nx = nx;
  args.xflags = xflags;
  args.cap = a.kmax + b.kmax;
  args.rows_vec = args.cap == 2 * K && aligned(out_xy, 16) && aligned(xflags, (uintptr_t)(2 * K));
  args.err = ctx->v.err;
  const bool fixed = a.nv == nullptr && b.nv == nullptr && a.kmax == K && b.kmax == K &&
                     args.a.vec4 && args.b.vec4 && args.rows_vec;
  return status_of(dgal::launch_intersect_fwd(args, K, fixed, static_cast<hipStream_t>(stream)));
}

int dgal_intersect_backward(dgal_ctx* ctx, dgal_polys a, dgal_polys b, const float* grad_xy,
                            const uint8_t* nx, const uint8_t* xflags, float* grad_a_xy,
                            float* grad_b_xy, void* stream) {
  if (ctx == nullptr || !valid_polys(a) || !valid_polys(b)) return DGAL_EINVAL;
  if (a.count != b.count) return DGAL_EINVAL;
  if (a.count == 0) return DGAL_OK;
  if (grad_xy == nullptr || nx == nullptr || xflags == nullptr || grad_a_xy == nullptr ||
      grad_b_xy == nullptr)
    return DGAL_EINVAL;
  if (!aligned(grad_xy, 8) || !aligned(grad_a_xy, 8) || !aligned(grad_b_xy, 8)) return DGAL_EINVAL;
  DeviceGuard g(ctx->v.device);
  if (!g.ok) return DGAL_EHIP;
  const int K = reg_k(a.kmax, b.kmax);
  dgal::IntersectBwdArgs args;
  args.a = poly_args(a, K);
  args.b = poly_args(b, K);
  args.grad_xy = grad_xy;
  args.nx = nx;
  args.xflags = xflags;
  args.cap = a.kmax + b.kmax;
  args.ga_xy = grad_a_xy;
  args.gb_xy = grad_b_xy;
  const bool fixed = a.nv == nullptr && b.nv == nullptr && a.kmax == K && b.kmax == K &&
                     args.a.vec4 && args.b.vec4;
  return status_of(dgal::launch_intersect_bwd(args, K, fixed, static_cast<hipStream_t>(stream)));
}

int dgal_area(dgal_ctx* ctx, dgal_polys p, float* area, void* stream) {
  if (ctx == nullptr || !valid_polys(p)) return DGAL_EINVAL;
  if (p.count == 0) return DGAL_OK;
  if (area == nullptr) return DGAL_EINVAL;
  DeviceGuard g(ctx->v.device);
  if (!g.ok) return DGAL_EHIP;
  const int K = p.kmax <= 4 ? 4 : 8;
  const dgal::PolyArgs pa = poly_args(p, K);
  const bool fixed = p.nv == nullptr && p.kmax == K && pa.vec4;
  return status_of(
      dgal::launch_area(pa, nullptr, area, K, fixed, false, static_cast<hipStream_t>(stream)));
}

int dgal_area_backward(dgal_ctx* ctx, dgal_polys p, const float* grad_area, float* grad_xy,
                       void* stream) {
  if (ctx == nullptr || !valid_polys(p)) return DGAL_EINVAL;
  if (p.count == 0) return DGAL_OK;
  if (grad_area == nullptr || grad_xy == nullptr || !aligned(grad_xy, 8)) return DGAL_EINVAL;
  DeviceGuard g(ctx->v.device);
  if (!g.ok) return DGAL_EHIP;
  const int K = p.kmax <= 4 ? 4 : 8;
  const dgal::PolyArgs pa = poly_args(p, K);
  const bool fixed = p.nv == nullptr && p.kmax == K && pa.vec4;
  return status_of(dgal::launch_area(pa, grad_area, grad_xy, K, fixed, true,
                                     static_cast<hipStream_t>(stream)));
}

}  // extern "C"

namespace {

bool valid_boxes(const dgal_boxes& a, const dgal_boxes& b) {
  if (a.count < 0 || a.count != b.count || a.dim != b.dim || (a.dim != 5 && a.dim != 7))
    return false;
  if (a.count > 0 && (a.p == nullptr || b.p == nullptr || !aligned(a.p, 4) || !aligned(b.p, 4)))
    return false;
  return true;
}

}  // namespace

extern "C" {

int dgal_iou_boxes(dgal_ctx* ctx, dgal_boxes a, dgal_boxes b, float* iou, uint8_t* nx,
                   uint8_t* xflags, void* stream) {
  if (ctx == nullptr || !valid_boxes(a, b)) return DGAL_EINVAL;
  if ((nx == nullptr) != (xflags == nullptr)) return DGAL_EINVAL;
  if (a.count == 0) return DGAL_OK;
  if (iou == nullptr || (xflags != nullptr && !aligned(xflags, 8))) return DGAL_EINVAL;
  DeviceGuard g(ctx->v.device);
  if (!g.ok) return DGAL_EHIP;
  dgal::BoxesFwdArgs args;
  args.a = a.p;
  args.b = b.p;
  args.count = a.count;
  args.iou = iou;
  args.nx = nx;
  args.xflags = xflags;
  args.err = ctx->v.err;
  return status_of(dgal::launch_boxes_fwd(args, a.dim == 7, nx != nullptr,
                                          static_cast<hipStream_t>(stream)));
}

int dgal_iou_boxes_backward(dgal_ctx* ctx, dgal_boxes a, dgal_boxes b, const float* grad_iou,
                            const uint8_t* nx, const uint8_t* xflags, float* grad_a,
                            float* grad_b, void* stream) {
  if (ctx == nullptr || !valid_boxes(a, b)) return DGAL_EINVAL;
  if (a.count == 0) return DGAL_OK;
  if (grad_iou == nullptr || nx == nullptr || xflags == nullptr || grad_a == nullptr ||
      grad_b == nullptr || !aligned(xflags, 8) || !aligned(grad_a, 4) || !aligned(grad_b, 4))
    return DGAL_EINVAL;
  DeviceGuard g(ctx->v.device);
  if (!g.ok) return DGAL_EHIP;
  dgal::BoxesBwdArgs args;
  args.a = a.p;
  args.b = b.p;
  args.count = a.count;
  args.grad = grad_iou;
  args.nx = nx;
  args.xflags = xflags;
  args.ga = grad_a;
  args.gb = grad_b;
  return status_of(dgal::launch_boxes_bwd(args, a.dim == 7, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
