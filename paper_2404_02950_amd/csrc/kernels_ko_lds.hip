// Per-stage kernels with Kreiss-Oliger dissipation (orders 2 and 3) on block-row tiles
// (boxes at least 64 cells wide), for every Laplacian order, instantiated from
// sh_stage.h: psi and Pi are both staged through LDS with the wider of the two radii.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_internal.h"
#include "sh_launch.h"
#include "sh_device.h"
#include "sh_stage.h"

#pragma clang fp contract(off)

namespace {

template <typename T, bool NT, int ROWS, int H, int KD>
void ko_lds2(int s, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  const dim3 grid(ntiles), block(SH_WAVE * ROWS);
  switch (s) {
    case 0: hipLaunchKernelGGL((k_stage_lds<T, 0, NT, ROWS, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    case 1: hipLaunchKernelGGL((k_stage_lds<T, 1, NT, ROWS, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    case 2: hipLaunchKernelGGL((k_stage_lds<T, 2, NT, ROWS, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    case 3: hipLaunchKernelGGL((k_stage_lds<T, 3, NT, ROWS, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    case 4: hipLaunchKernelGGL((k_stage_lds<T, 4, NT, ROWS, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    case 5: hipLaunchKernelGGL((k_stage_lds<T, 5, NT, ROWS, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
    default: hipLaunchKernelGGL((k_stage_lds<T, 6, NT, ROWS, H, KD>), grid, block, 0, st, tiles, ntiles, boxes); break;
  }
}

template <typename T, bool NT, int ROWS, int KD>
void ko_lds1(int s, int order, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  if (order == 1) ko_lds2<T, NT, ROWS, 1, KD>(s, tiles, ntiles, boxes, st);
  else if (order == 2) ko_lds2<T, NT, ROWS, 2, KD>(s, tiles, ntiles, boxes, st);
  else ko_lds2<T, NT, ROWS, 3, KD>(s, tiles, ntiles, boxes, st);
}

template <typename T, bool NT>
void ko_lds0(int s, int kind, int order, int ko, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  if (kind == 4) {
    if (ko == 2) ko_lds1<T, NT, 4, 2>(s, order, tiles, ntiles, boxes, st);
    else ko_lds1<T, NT, 4, 3>(s, order, tiles, ntiles, boxes, st);
  } else {
    if (ko == 2) ko_lds1<T, NT, 8, 2>(s, order, tiles, ntiles, boxes, st);
    else ko_lds1<T, NT, 8, 3>(s, order, tiles, ntiles, boxes, st);
  }
}

}  // namespace

void sh_launch_stage_ko_lds(int prec, int s, int kind, bool nt, int order, int ko, const Tile* tiles, int ntiles,
                            const BoxDev* boxes, hipStream_t st) {
  if (ntiles == 0) return;
  if (prec == 0) {
    if (nt) ko_lds0<double, true>(s, kind, order, ko, tiles, ntiles, boxes, st);
    else ko_lds0<double, false>(s, kind, order, ko, tiles, ntiles, boxes, st);
  } else {
    if (nt) ko_lds0<float, true>(s, kind, order, ko, tiles, ntiles, boxes, st);
    else ko_lds0<float, false>(s, kind, order, ko, tiles, ntiles, boxes, st);
  }
}
