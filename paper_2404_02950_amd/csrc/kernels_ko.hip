// Per-stage kernels with Kreiss-Oliger dissipation (orders 2 and 3) on wave-row tiles
// (boxes narrower than 64 cells; the dissipation stencils Pi as well, whose neighbours are
// read through the caches), and the right-hand-side kernels, for every Laplacian order,
// instantiated from sh_stage.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_internal.h"
#include "sh_launch.h"
#include "sh_device.h"
#include "sh_stage.h"

#pragma clang fp contract(off)

namespace {

template <typename T, bool NT, int H, int KD>
void ko_stage2(int s, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  const dim3 grid((ntiles + SH_BLOCK / SH_WAVE - 1) / (SH_BLOCK / SH_WAVE)), block(SH_BLOCK);
  switch (s) {
    case 0: hipLaunchKernelGGL((k_stage<T, 0, NT, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    case 1: hipLaunchKernelGGL((k_stage<T, 1, NT, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    case 2: hipLaunchKernelGGL((k_stage<T, 2, NT, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    case 3: hipLaunchKernelGGL((k_stage<T, 3, NT, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    case 4: hipLaunchKernelGGL((k_stage<T, 4, NT, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    case 5: hipLaunchKernelGGL((k_stage<T, 5, NT, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    default: hipLaunchKernelGGL((k_stage<T, 6, NT, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
  }
}

template <typename T, bool NT, int KD>
void ko_stage1(int s, int order, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  if (order == 1) ko_stage2<T, NT, 1, KD>(s, tiles, ntiles, boxes, st);
  else if (order == 2) ko_stage2<T, NT, 2, KD>(s, tiles, ntiles, boxes, st);
  else ko_stage2<T, NT, 3, KD>(s, tiles, ntiles, boxes, st);
}

template <typename T, bool NT>
void ko_stage0(int s, int order, int ko, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  if (ko == 2) ko_stage1<T, NT, 2>(s, order, tiles, ntiles, boxes, st);
  else ko_stage1<T, NT, 3>(s, order, tiles, ntiles, boxes, st);
}

template <typename T, int KD>
void ko_rhs1(int order, const Tile* tiles, int ntiles, const BoxDev* boxes, const long long* out_off, double* out,
             hipStream_t st) {
  const dim3 grid((ntiles + SH_BLOCK / SH_WAVE - 1) / (SH_BLOCK / SH_WAVE)), block(SH_BLOCK);
  if (order == 1) hipLaunchKernelGGL((k_rhs<T, 1, KD>), grid, block, 0, st, tiles, ntiles, boxes, out_off, out);
  else if (order == 2) hipLaunchKernelGGL((k_rhs<T, 2, KD>), grid, block, 0, st, tiles, ntiles, boxes, out_off, out);
  else hipLaunchKernelGGL((k_rhs<T, 3, KD>), grid, block, 0, st, tiles, ntiles, boxes, out_off, out);
}

}  // namespace

void sh_launch_stage_ko(int prec, int s, bool nt, int order, int ko, const Tile* tiles, int ntiles,
                        const BoxDev* boxes, hipStream_t st) {
  if (ntiles == 0) return;
  if (prec == 0) {
    if (nt) ko_stage0<double, true>(s, order, ko, tiles, ntiles, boxes, st);
    else ko_stage0<double, false>(s, order, ko, tiles, ntiles, boxes, st);
  } else {
    if (nt) ko_stage0<float, true>(s, order, ko, tiles, ntiles, boxes, st);
    else ko_stage0<float, false>(s, order, ko, tiles, ntiles, boxes, st);
  }
}

void sh_launch_rhs_ko(int prec, int order, int ko, const Tile* tiles, int ntiles, const BoxDev* boxes,
                      const long long* out_off, double* out, hipStream_t st) {
  if (ntiles == 0) return;
  if (prec == 0) {
    if (ko == 2) ko_rhs1<double, 2>(order, tiles, ntiles, boxes, out_off, out, st);
    else ko_rhs1<double, 3>(order, tiles, ntiles, boxes, out_off, out, st);
  } else {
    if (ko == 2) ko_rhs1<float, 2>(order, tiles, ntiles, boxes, out_off, out, st);
    else ko_rhs1<float, 3>(order, tiles, ntiles, boxes, out_off, out, st);
  }
}
