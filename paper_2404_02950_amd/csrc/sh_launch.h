// Host-side launch wrappers of the kernels in kernels.hip (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_internal.h"

// order: the Laplacian order of appendix A (1, 2, 3: 7-, 13-, 19-point stencil); ko:
// the Kreiss-Oliger dissipation order (0 = off, 2, 3); kind: 0 = wave-row tiles, 4 or 8 =
// block-row tiles of that many rows
void sh_launch_stage(int prec, int s, int kind, bool nt, int order, int ko, const Tile* tiles, int ntiles,
                     const BoxDev* boxes, hipStream_t st);
void sh_launch_rhs(int prec, int order, int ko, const Tile* tiles, int ntiles, const BoxDev* boxes,
                   const long long* out_off, double* out, hipStream_t st);
// with dissipation (kernels_ko.hip: wave rows; kernels_ko_lds.hip: block rows)
void sh_launch_stage_ko(int prec, int s, bool nt, int order, int ko, const Tile* tiles, int ntiles,
                        const BoxDev* boxes, hipStream_t st);
void sh_launch_stage_ko_lds(int prec, int s, int kind, bool nt, int order, int ko, const Tile* tiles, int ntiles,
                            const BoxDev* boxes, hipStream_t st);
void sh_launch_rhs_ko(int prec, int order, int ko, const Tile* tiles, int ntiles, const BoxDev* boxes,
                      const long long* out_off, double* out, hipStream_t st);
// orders 2 and 3 (kernels_hilap.hip)
void sh_launch_stage_hilap(int prec, int s, int kind, bool nt, int order, const Tile* tiles, int ntiles,
                           const BoxDev* boxes, hipStream_t st);
void sh_launch_rhs_hilap(int prec, int order, const Tile* tiles, int ntiles, const BoxDev* boxes,
                         const long long* out_off, double* out, hipStream_t st);
void sh_launch_counter_inc(LevelScal* ls, int n, hipStream_t st);
void sh_launch_counter_zero(LevelScal* ls, int n, hipStream_t st);
void sh_launch_counter_inc_list(LevelScal* const* ls, int n, hipStream_t st);
// chunks of up to SH_WAVE cells (one wavefront each)
void sh_launch_ghost_copy(int prec, const CopySeg* segs, const SegBlock* chunks, int nchunks, const BoxDev* boxes,
                          int role, int ncomp, hipStream_t st);
// interp: 1 = linear conservative, 4 = quartic conservative
void sh_launch_ghost_interp(int prec, int interp, const InterpSeg* segs, const SegBlock* blocks, int nblocks,
                            const BoxDev* fboxes, const BoxDev* cboxes, int role, int anum, int ncomp,
                            hipStream_t st);
void sh_launch_avgdown(int prec, const AvgSeg* segs, const SegBlock* blocks, int nblocks, const BoxDev* cboxes,
                       const BoxDev* fboxes, double* tee, int tee_nc, long long tee_cs, int write_coarse,
                       hipStream_t st);
void sh_launch_regrid_copy(int prec, const CopySeg* segs, const SegBlock* blocks, int nblocks, const BoxDev* dboxes,
                           const BoxDev* sboxes, const double* tee_src, double* tee_dst, int tee_nc,
                           long long tee_cs_src, long long tee_cs_dst, hipStream_t st);
void sh_launch_tag(int prec, const Tile* tiles, int ntiles, const BoxDev* boxes, uint8_t* mask, int* tile_count,
                   const double* tee, const TeeSpec& te, int mode, hipStream_t st);
// max |U_c| over the valid cells of a level's tiles: one partial per tile (4 doubles),
// then the maximum over the tiles into out[4]
void sh_launch_absmax(int prec, const Tile* tiles, int ntiles, const BoxDev* boxes, double* part, double* out,
                      hipStream_t st);
void sh_launch_scan(const int* in, long long* out, int n, hipStream_t st);
void sh_launch_tag_compact(const Tile* tiles, int ntiles, const BoxDev* boxes, const uint8_t* mask,
                           const long long* tile_off, int* idx, long long cap, hipStream_t st);
void sh_launch_tag_octants(const Tile* tiles, int ntiles, const BoxDev* boxes, const uint8_t* mask, int halve, int r,
                           int bsh, int nb, unsigned long long* oct, long long nwords, hipStream_t st);
void sh_launch_energy(int prec, const Tile* tiles, int ntiles, const BoxDev* boxes, const uint8_t* covered,
                      EnergyPartial* part, hipStream_t st);
void sh_launch_energy_final(const EnergyPartial* part, int n, double vol, double* out, hipStream_t st);
void sh_launch_mark_covered(const AvgSeg* segs, const SegBlock* blocks, int nblocks, const BoxDev* cboxes,
                            uint8_t* covered, hipStream_t st);
void sh_launch_xfer(int prec, bool to_box, const BoxDev* boxes, const long long* off, int nbox, double* stage, int role,
                    int g, long long total, hipStream_t st);
void sh_launch_debug_scalars(const LevelScal* ls, int s, double* out, hipStream_t st);
void sh_launch_fused(int prec, bool nt, int shape, int variant, int nst, const Tile* tiles, int ntiles,
                     const BoxDev* boxes, hipStream_t st);
void sh_fused_footprint(int shape, int* tx, int* ty);
// streaming probes (kernels_stream.hip): kind 0 = read, 1 = write, 2 = copy of nwords
// 16-byte words
void sh_launch_stream(int kind, const void* src, void* dst, long long nwords, hipStream_t st);
long long sh_stream_words_per_block();
// debug: NaN into the ghost shell (ng deep, first ncomp components) of buffer `role` of
// every box; nplanes = the deepest box's nz + 2 ng
void sh_launch_poison_ghosts(int prec, const BoxDev* boxes, int nboxes, int nplanes, int ng, int role, int ncomp,
                             hipStream_t st);

