// Per-stage kernels with the higher-order Laplacians of appendix A (order 2: 13-point,
// order 3: 19-point stencil), instantiated from sh_stage.h in a translation unit of their
// own so they compile alongside the order-1 kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_internal.h"
#include "sh_launch.h"
#include "sh_device.h"
#include "sh_stage.h"

#pragma clang fp contract(off)

void sh_launch_stage_hilap(int prec, int s, int kind, bool nt, int order, const Tile* tiles, int ntiles,
                           const BoxDev* boxes, hipStream_t st) {
  if (order == 2) stage_launch_radius<2>(prec, s, kind, nt, tiles, ntiles, boxes, st);
  else stage_launch_radius<3>(prec, s, kind, nt, tiles, ntiles, boxes, st);
}

void sh_launch_rhs_hilap(int prec, int order, const Tile* tiles, int ntiles, const BoxDev* boxes,
                         const long long* out_off, double* out, hipStream_t st) {
  if (order == 2) rhs_launch_radius<2>(prec, tiles, ntiles, boxes, out_off, out, st);
  else rhs_launch_radius<3>(prec, tiles, ntiles, boxes, out_off, out, st);
}
