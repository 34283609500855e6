// device_stubs.cpp -- stand-ins for the kernel translation units in the
// sanitizer build of the library's host code (abi_host.c): that build has no
// GPU code, and without a device no call may reach a launcher, so each stub
// reports and aborts.
#include <stdio.h>
#include <stdlib.h>

#include "../../paper_2011_11134_amd/csrc/internal.hpp"

namespace dgal {

[[noreturn]] static void reached(const char* what) {
  fprintf(stderr, "device layer reached without a device: %s\n", what);
  abort();
}

int matrix_forward(const CtxView&, dgal_polys, dgal_polys, const int64_t*, const int64_t*,
                   const int64_t*, int, int, float*, int64_t, dgal_saved*, hipStream_t,
                   const LaunchShape&) {
  reached("matrix_forward");
}
int matrix_backward(const CtxView&, dgal_polys, dgal_polys, const int64_t*, const int64_t*,
                    const int64_t*, int, int, const float*, int64_t, const dgal_saved*, float*,
                    float*, float*, float*, hipStream_t, const LaunchShape&) {
  reached("matrix_backward");
}
int matrix_scratch_init(int) { reached("matrix_scratch_init"); }
int matrix_forward_noalloc(const CtxView&, dgal_polys, dgal_polys, const int64_t*,
                           const int64_t*, const int64_t*, int, int, float*, int64_t, hipStream_t,
                           const LaunchShape&) {
  reached("matrix_forward_noalloc");
}
hipError_t launch_pairs_fwd(const PairsFwdArgs&, int, bool, bool, bool, hipStream_t,
                            const LaunchShape&) {
  reached("launch_pairs_fwd");
}
hipError_t launch_pairs_bwd(const PairsBwdArgs&, int, bool, bool, hipStream_t,
                            const LaunchShape&) {
  reached("launch_pairs_bwd");
}
hipError_t launch_intersect_fwd(const IntersectArgs&, int, bool, hipStream_t) {
  reached("launch_intersect_fwd");
}
hipError_t launch_intersect_bwd(const IntersectBwdArgs&, int, bool, hipStream_t) {
  reached("launch_intersect_bwd");
}
hipError_t launch_area(const PolyArgs&, const float*, float*, int, bool, bool, hipStream_t) {
  reached("launch_area");
}
hipError_t launch_boxes_fwd(const BoxesFwdArgs&, bool, bool, hipStream_t) {
  reached("launch_boxes_fwd");
}
hipError_t launch_boxes_bwd(const BoxesBwdArgs&, bool, hipStream_t) {
  reached("launch_boxes_bwd");
}
hipError_t launch_simple_fwd(const SimpleFwdArgs&, int, hipStream_t) {
  reached("launch_simple_fwd");
}
hipError_t launch_simple_bwd(const SimpleBwdArgs&, int, hipStream_t) {
  reached("launch_simple_bwd");
}
hipError_t launch_validate(const PolyArgs&, uint8_t*, int64_t*, bool, hipStream_t) {
  reached("launch_validate");
}

}  // namespace dgal
