/*
 * shamr.h -- C-ABI of libshamr: the per-level AMR time step of a two-component scalar
 * field (axion strings) on one AMD Instinct MI355X (gfx950).
 *
 * Paper: M. Buschmann, "sledgehamr: Simulating scalar fields with adaptive mesh
 * refinement", arXiv:2404.02950.  The problem solved (section "Minimal example",
 * eqs. EOM1/EOM2): on a periodic cube of n0^3 coarse cells of side L,
 *
 *     d psi_i / d eta = Pi_i
 *     d Pi_i  / d eta = lap psi_i - (alpha/eta) Pi_i - lambda eta^beta psi_i (psi1^2 + psi2^2 - 1)
 *
 * (the paper's example has alpha = 2, beta = 2, lambda = 1), discretised with the
 * Laplacian of appendix A (order 1, 2 or 3: the 7-, 13- or 19-point stencil) and
 * classic RK4 or SSPRK3 (appendix E, integrator types 4 and 3/10) on a
 * block-structured hierarchy of levels with dx_l = (L/n0)/2^l and
 * dt_l = cfl * dx_l (section II, eq. dtscaling), advanced by Berger-Oliger subcycling
 * (section II.A, Fig. 2).
 *
 * Conventions
 * -----------
 * - Box: six int32 (x_lo, y_lo, z_lo, x_hi, y_hi, z_hi), inclusive, in the index space of
 *   its level ([0, n0*2^l) per axis).  Boxes of a level are disjoint; boxes of a level
 *   l >= 1 have even lo and odd hi.
 * - Dense state arrays exchanged with the library are float64, laid out box after box
 *   (in the order given to sh_set_level_layout), each box as [comp][z][y][x] with
 *   comp = (psi1, psi2, Pi1, Pi2), x fastest; with_ghosts = 1 adds the one-cell ghost
 *   shell, i.e. (nz+2)(ny+2)(nx+2) values per component.
 * - Buffer roles: 0 = U_n (the current state of the level), 1 and 2 = the RK stage
 *   states, 3 = the state before the last step of the level (the "old" coarse state
 *   used by time interpolation).
 * - Every call returns an sh_status and never throws or aborts across the ABI; after a
 *   non-OK status, sh_last_error() gives a message (thread-local).
 * - All device work is queued asynchronously on the HIP stream given at creation.  Calls
 *   that return host data (sh_tag_cells, sh_energy, sh_read_state to host, sh_sync)
 *   synchronise that stream and report kernel failures as SH_EDEVICE.
 * - One handle must not be used from two threads at once.
 * - Device memory for the fields is owned by the caller: one arena per level, sized by
 *   sh_arena_bytes, kept alive until the level's next layout or sh_hierarchy_destroy.
 *   The library allocates only its small index tables (at layout time), never on the
 *   stepping path.
 */
#ifndef SHAMR_H
#define SHAMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sh_hierarchy_s* sh_hierarchy;
typedef struct sh_batch_s* sh_batch;
typedef struct sh_graph_s* sh_graph;  /* a recorded sequence of level steps (HIP graph) */

typedef enum {
  SH_OK = 0,
  SH_EINVAL = 1,  /* bad argument or layout */
  SH_ENOMEM = 2,  /* arena too small / host or table allocation failed */
  SH_ENEST = 3,   /* a fine level is not properly nested in its coarse level */
  SH_ESTATE = 4,  /* call not valid in the current state (e.g. no layout yet) */
  SH_EDEVICE = 5  /* a HIP call or kernel failed */
} sh_status;

typedef enum { SH_F64 = 0, SH_F32 = 1 } sh_prec;

typedef struct {
  int32_t n0;           /* coarse cells per axis (amr.coarse_level_grid_size) */
  double L;             /* box length (sim.L) */
  double cfl;           /* dt_l / dx_l (sim.cfl) */
  double eta0;          /* start time (sim.t_start); level time = eta0 + k_l * dt_l */
  double lambda;        /* potential strength */
  double alpha_fric;    /* friction coefficient: the -(alpha/eta) Pi term */
  int32_t beta_pot;     /* potential time exponent, >= 0: lambda * eta^beta */
  int32_t max_level;    /* finest level allowed (amr.max_refinement_levels) */
  int32_t blocking_factor;  /* box sides are multiples of it (amr.blocking_factor) */
  int32_t max_box;      /* largest box side produced by sh_cluster_tags */
  int32_t n_error_buf;  /* tag buffer width in cells (amr.n_error_buf) */
  int32_t prec;         /* sh_prec: SH_F64, or SH_F32 = float32 storage and stencil,
                           float64 time, accumulator and reductions */
  int32_t integrator;   /* integrator.type of appendix E: 4 (or 0) = classic RK4;
                           3 or 10 = SSPRK3, the three-stage strong-stability-preserving
                           method (both run its Shu-Osher form in three state buffers and
                           no accumulator, so sh_arena_bytes is smaller); 21 = RKN4, read
                           as Nystrom's classical three-stage fourth-order method for
                           psi'' = a(psi) (appendices B and D use it).  It applies only
                           when the acceleration does not depend on Pi: alpha_fric must
                           be 0 and ko_order 0 (SH_EINVAL otherwise); it keeps RK4's
                           float64 accumulator and is not fused on level 0; 22 = RKN5,
                           read as a four-stage fifth-order Nystrom tableau (appendix B),
                           with RKN4's restrictions, on single periodic levels only
                           (max_level 0; no shadow level, no batching, not fused) */
  int32_t lap_order;    /* Laplacian order of appendix A (the minimal example's `order`):
                           1 (or 0) = 7-point, 2 = 13-point, 3 = 19-point stencil.  The
                           ghost shell of refined levels is that many cells deep (and so
                           is every ghost fill between stages); the fused step needs 1 */
  int32_t interp;       /* amr.interpolation_type of appendix E for ghost cells and new fine
                           cells: 1 (or 0) = linear conservative, 4 = quartic conservative
                           (the paper's default; tensor product of the 1-D conservative
                           quartic through five coarse averages).  Quartic interpolation
                           reads two coarse cells beyond each parent: refined levels then
                           keep at least two ghost layers, and nesting needs that margin */
  int32_t ko_order;     /* sim.dissipation_order (section II, Kreiss-Oliger dissipation):
                           0 = off, 2 or 3 = the ghost cells the operator needs, read as
                           p = 3 or 5: Q = (-1)^((p+3)/2) eps dx^p / 2^(p+1) times the sum
                           of the (p+1)-st central differences, added to the right-hand
                           side of all four components.  Refined levels then keep that
                           many ghost layers, the fills between stages carry Pi too, the
                           block-row stage kernel stages Pi through LDS as well, and the
                           fused step is not used */
  double ko_eps;        /* sim.dissipation_strength eps >= 0 */
  int32_t tee_fields;   /* truncation error estimates kept per cell (Sec. IV.C): 0 = one,
                           the maximum over the four components; 1 = one per component,
                           so that each field can have its own threshold and modifier
                           (sh_set_tee_fields); arenas then hold 32 instead of 8 bytes of
                           estimates per valid cell */
} sh_params;

/* Device bytes needed for the arena of a level with the given boxes (section II: a
   level is a union of boxes; per box the four fields of eqs. EOM1/EOM2 in three state
   buffers, a float64 accumulator for RK4, and the ghost shell the stencil needs).  The
   caller allocates it; the library keeps no field storage of its own.  Returns 0 for
   invalid arguments. */
size_t sh_arena_bytes(const sh_params* p, int32_t lev, int32_t nboxes, const int32_t* boxes);

/* Create a hierarchy for the problem of section "Minimal example" (eqs. EOM1/EOM2 on
   a periodic cube of n0^3 coarse cells of side L) with the simulation and AMR
   parameters of appendix E (sim.L, sim.cfl, sim.t_start, amr.max_refinement_levels,
   amr.blocking_factor, amr.n_error_buf, integrator.type, interpolation type) carried in
   sh_params; the handle is host memory owned by the library until
   sh_hierarchy_destroy.  `hip_stream` is a hipStream_t (NULL = default stream) that all
   device work of this hierarchy is queued on.  Errors: SH_EINVAL (n0 < 1, L or cfl not
   positive, beta < 0, max_level < 0 or > 15, blocking_factor < 2, prec not 0/1,
   integrator not 0, 3, 4, 10, 21 or 22, RKN4/RKN5 with friction or dissipation, RKN5 with
   max_level > 0, lap_order not 0..3, interp not 0, 1 or 4, ko_order not 0, 2 or 3,
   ko_eps negative or not finite), SH_EDEVICE (no HIP device). */
sh_status sh_hierarchy_create(const sh_params* p, void* hip_stream, sh_hierarchy* out);

/* Set, change or remove the box layout of level `lev` (section II: boxes whose sides
   are multiples of the blocking factor; section II.C: proper nesting).
   - lev == 0: the boxes must tile the whole periodic domain.  Values are unset until
     sh_write_state (unless a previous level-0 layout existed: its values are kept).
   - lev == number of levels (a new level): valid cells are interpolated from level
     lev-1 (sh_params.interp, all 4 components) and the ghost cells filled; the level
     starts at the time of level lev-1.
   - an existing level: cells valid in the old layout keep their values, the others are
     interpolated from level lev-1 (a regrid); ghosts are refilled.
   - nboxes == 0 removes level lev and every finer level.
   `arena` is caller-owned device memory of at least sh_arena_bytes(...) bytes; the old
   arena of the level must stay valid until the work queued by this call has run.
   Errors: SH_EINVAL (bad box, overlap, level 0 not covering, lev > max_level or
   > number of levels), SH_ENOMEM (arena too small), SH_ENEST (not nested in lev-1). */
sh_status sh_set_level_layout(sh_hierarchy h, int32_t lev, int32_t nboxes, const int32_t* boxes,
                              void* arena, size_t arena_bytes);

/* Copy a dense float64 state (layout above) of the four fields psi1, psi2, Pi1, Pi2
   (section "Minimal example": the two scalars and their conformal-time derivatives)
   into buffer role `role` of level `lev`; values are rounded to the storage precision.
   `src` is host memory (src_is_device = 0, the call copies it before returning) or
   device memory (queued on the stream).  Errors: SH_EINVAL, SH_ESTATE (no layout). */
sh_status sh_write_state(sh_hierarchy h, int32_t lev, int32_t role, const double* src, int32_t src_is_device,
                         int32_t with_ghosts);

/* Copy buffer role `role` of level `lev` out as a dense float64 state of the four
   fields of section "Minimal example" (layout above).  `dst` is host memory (the call
   synchronises the stream and reports kernel failures as SH_EDEVICE) or device memory
   (queued).  Errors: SH_EINVAL, SH_ESTATE (no layout). */
sh_status sh_read_state(sh_hierarchy h, int32_t lev, int32_t role, double* dst, int32_t dst_is_device,
                        int32_t with_ghosts);

/* Ghost fill of the psi components of buffer `role` of level `lev` (section II.A): copies
   from the level's own boxes and periodic images, then, for lev >= 1, the remaining
   ghost cells (as deep as the Laplacian order) by linear or quartic conservative
   interpolation (appendix E, interpolation type 1 or 4, sh_params.interp) of the coarse
   states at the start (role 3) and end (role 0) of the coarse step, linear in time with
   alpha = alpha_num / 4 in [0, 4]. */
sh_status sh_fill_ghosts(sh_hierarchy h, int32_t lev, int32_t role, int32_t alpha_num);

/* One integrator step of level `lev` by dt_lev (section II.A, Fig. 2): stage 1, then
   ghost fill and stage for the remaining stages (alpha = (substep + c_s)/2 with
   c = (0, 1/2, 1/2, 1) for RK4 and (0, 1, 1/2) for SSPRK3), then the same-level ghost
   copy of the new state and, for lev >= 1 and substep == 0, its coarse/fine ghost fill
   at alpha = 1/2 (a substep-1 step ends in the synchronisation, sh_average_down).
   `substep` in {0, 1} is which half of the parent's step this is (ignored for lev 0).
   Does not recurse into finer levels: the caller composes the subcycling order. */
sh_status sh_advance_level(sh_hierarchy h, int32_t lev, int32_t substep);

/* Synchronisation of levels fine_lev and fine_lev-1 (section II.A): average the fine
   level's 2x2x2 children onto every covered coarse cell (all components), refresh the
   coarse level's same-level ghosts, then refill the fine ghosts with no temporal
   interpolation (alpha = 1).  Both levels must be at the same time. */
sh_status sh_average_down(sh_hierarchy h, int32_t fine_lev);

/* Problem-specific tagging (section "Problem-specific cell tagging"): a valid cell of
   level `lev` is tagged iff the phase of psi1 + i psi2 winds around any of its 12
   incident plaquettes (crossing-number rule).  Fills the level's ghosts first.
   Writes `mask_dev` (device, one byte per valid cell in the dense box order, may be
   NULL), and up to `cap` tagged cells as global (x, y, z) int32 triplets to host
   `idx_host` (may be NULL); `*ntag` receives the total count.  Synchronises. */
sh_status sh_tag_cells(sh_hierarchy h, int32_t lev, uint8_t* mask_dev, int32_t* idx_host, int64_t cap,
                       int64_t* ntag);

/* sh_tag_cells for callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same tagging, mask
   and list, but the compacted list is staged in a fixed device array of the library
   (1048576 cells = 12 MiB, held by every device the library runs on until the process
   ends) instead of a buffer it grows with hipMalloc; the call makes no allocation.
   Errors as sh_tag_cells, plus SH_EINVAL when idx_host is given with cap above 1048576.
   The array is shared by every call on a device: calls that overlap on one device (from
   several threads or streams) race; each call leaves its list there. */
sh_status sh_tag_cells_noalloc(sh_hierarchy h, int32_t lev, uint8_t* mask_dev, int32_t* idx_host, int64_t cap,
                               int64_t* ntag);

/* Composite energy over all levels, counting only cells not covered by a finer level
   (appendix B's convergence measure for this field): e_host[4] = {kinetic, gradient,
   potential, total}, float64, with forward-difference gradients and potential
   lambda eta^beta / 4 (|psi|^2 - 1)^2.  `nonfinite` (may be NULL) receives the number
   of counted cells holding a non-finite value.  Synchronises. */
sh_status sh_energy(sh_hierarchy h, double* e_host, int64_t* nonfinite);

/* Right-hand side f(U_n) of eqs. EOM1/EOM2 at the level's current time, with the
   current ghost values, into device `out_dev` (dense float64 layout, no ghosts). */
sh_status sh_eval_rhs(sh_hierarchy h, int32_t lev, double* out_dev);

/* Level bookkeeping: steps taken, current time eta0 + k dt, boxes and valid cells. */
sh_status sh_level_info(sh_hierarchy h, int32_t lev, int64_t* k, double* eta, int32_t* nboxes, int64_t* ncells);

/* Number of levels with a layout. */
int32_t sh_num_levels(sh_hierarchy h);

/* Berger-Rigoutsos clustering on the host (section II.C, global regrid): from `ntag`
   tagged cells of level `lev` (global (x, y, z) triplets) produce boxes of level lev+1
   that cover the tags grown by n_error_buf cells, with sides multiples of the blocking
   factor and at most max_box, properly nested in level lev's current layout (tags
   whose refinement would break nesting are dropped).  Writes at most `cap` boxes to
   `boxes_out` (6 int32 each) and the count to `*nboxes`; SH_ENOMEM if cap is too small
   (the count is still written). */
sh_status sh_cluster_tags(sh_hierarchy h, int32_t lev, int64_t ntag, const int32_t* tags, double efficiency,
                          int32_t* boxes_out, int32_t cap, int32_t* nboxes);

/* The same clustering without a hierarchy (host only, needs no GPU): tags of a level of
   M^3 cells whose layout is `level_boxes` (nlevel_boxes == 0: the level covers the whole
   domain, as level 0 does). */
sh_status sh_cluster_boxes(int32_t M, int32_t nlevel_boxes, const int32_t* level_boxes, int32_t blocking_factor,
                           int32_t max_box, int32_t n_error_buf, double efficiency, int64_t ntag,
                           const int32_t* tags, int32_t* boxes_out, int32_t cap, int32_t* nboxes);

/* Clustering with the tags of the next finer level carried down (section II.B: every
   tagged cell is refined with its buffer; levels are rebuilt coarsest first, so level l's
   new boxes must already leave room for the refinement of level l+1's tags).  As
   sh_cluster_tags / sh_cluster_boxes, plus `ncarried` cells of level l+1 (x, y, z int32
   triples in its index space, 0 <= x < 2M) whose coarse parents (x / 2), grown by
   grow + n_error_buf cells (periodic), are clustered as if tagged; grow = 1 with
   n_error_buf = 2 makes the rebuilt level l+1 reach at least 6 of its cells past every
   carried tag (the tag's buffer of 2 and the nesting gap of half a blocking factor).
   The tag lists are read only and stay the caller's.  Errors: those of the plain
   calls, and SH_EINVAL for a carried cell outside level l+1's index space, ncarried < 0,
   grow < 0 or grow > M. */
sh_status sh_cluster_tags_carried(sh_hierarchy h, int32_t lev, int64_t ntag, const int32_t* tags, int64_t ncarried,
                                  const int32_t* carried, int32_t grow, double efficiency, int32_t* boxes_out,
                                  int32_t cap, int32_t* nboxes);
sh_status sh_cluster_boxes_carried(int32_t M, int32_t nlevel_boxes, const int32_t* level_boxes,
                                   int32_t blocking_factor, int32_t max_box, int32_t n_error_buf, double efficiency,
                                   int64_t ntag, const int32_t* tags, int64_t ncarried, const int32_t* carried,
                                   int32_t grow, int32_t* boxes_out, int32_t cap, int32_t* nboxes);

/* Clustering from tagged blocks instead of tag lists (section II.C, global regrid): for
   levels with many tags no list crosses to the host.  Clustering works on blocks of bf/2
   cells; the bitset of a level of M cells per axis has one bit per block, bit k = x +
   nb (y + nb z) of block (x, y, z), nb = M / (bf/2), in nwords = ceil(nb^3 / 64) uint64
   words owned by the caller.
   sh_tag_blocks: tags level `lev` on the GPU (as sh_tag_cells) and ORs into `bits_host`
   every block met by the cube [c - r, c + r] (periodic) around each tagged cell c: blocks
   of level lev (halve = 0; r = n_error_buf gives the blocks sh_cluster_tags marks for
   those tags) or of level lev - 1 (halve = 1, c replaced by its parent c / 2; r = grow +
   n_error_buf gives the blocks sh_cluster_tags_carried marks for carried tags).  With
   at least one tagged cell per 16 blocks (bf/2 a power of two, bf/4 <= r < bf/2), each
   tagged cell sets, on the GPU, the bit of its own block in the octant bitsets of the
   neighbours its cube reaches, and only those come to the host (8 nwords words), each
   grown there by one block towards its octant; otherwise the tag list comes to the host
   and is marked there.  *ntag (may be NULL) receives the
   number of tagged cells.  Synchronises.  Errors: SH_EINVAL (no such level, halve on
   level 0, r < 0, a null bitset or one of the wrong size), SH_ESTATE (stale level, or
   called during capture), SH_EDEVICE.
   sh_cluster_blocks: the boxes of level lev+1 from a bitset of level lev's blocks (the OR
   of sh_tag_blocks calls): the boxes sh_cluster_tags(_carried) gives for the tags that
   set those bits; output and errors as sh_cluster_tags, SH_EINVAL for a bitset of the
   wrong size.
   sh_cluster_boxes_bits is the same clustering without a hierarchy (host only; the
   level's layout as in sh_cluster_boxes), and sh_dilate_octants the host step of
   sh_tag_blocks: ORs into `bits` eight octant bitsets of nwords words each (one after
   the other; bit 0 of the octant index: the +x neighbour, else -x; bit 1: +y; bit 2:
   +z), each grown by one block towards its octant (periodic). */
sh_status sh_tag_blocks(sh_hierarchy h, int32_t lev, int32_t halve, int32_t r, uint64_t* bits_host, int64_t nwords,
                        int64_t* ntag);
sh_status sh_cluster_blocks(sh_hierarchy h, int32_t lev, const uint64_t* bits, int64_t nwords, double efficiency,
                            int32_t* boxes_out, int32_t cap, int32_t* nboxes);
sh_status sh_cluster_boxes_bits(int32_t M, int32_t nlevel_boxes, const int32_t* level_boxes,
                                int32_t blocking_factor, int32_t max_box, double efficiency, const uint64_t* bits,
                                int64_t nwords, int32_t* boxes_out, int32_t cap, int32_t* nboxes);
sh_status sh_dilate_octants(int32_t M, int32_t blocking_factor, const uint64_t* octants, uint64_t* bits,
                            int64_t nwords);

/* Local regrid (section II, "Local versus global regrid"): instead of clustering all tags
   anew, keep every box of the finer level and grow it, by whole blocks of the blocking
   factor bf, where tagged cells (with their n_error_buf buffer) reach past it; coarser
   levels grow where the added blocks need the nesting gap.  Host computations on box
   lists (the tags come from sh_tag_cells); the caller applies the result with
   sh_set_level_layout (old boxes + added ones, coarsest changed level first).
   sh_local_tag_boxes: boxes to add to a level of M_fine cells per axis, given its current
   boxes (none for a new level) and the tags (x, y, z int32 triples) of the level below;
   the blocks that meet the refinement of each cube [tag - n_error_buf, tag + n_error_buf]
   (periodic) and are not yet in the level.
   sh_local_nest_boxes: boxes to add to a level of M_level cells per axis so that the
   added boxes of the next finer level (added_fine, its index space) keep the nesting gap
   of bf/2 cells of this level.
   Added blocks are merged into runs along x of at most max_box cells, listed in (z, y, x)
   block order; *nboxes receives their number.  Errors: SH_EINVAL (boxes not made of whole
   blocks inside the level, a tag outside the coarser level, bad sizes), SH_ENOMEM (cap too
   small; *nboxes is still set). */
sh_status sh_local_tag_boxes(int32_t M_fine, int32_t nfine, const int32_t* fine_boxes, int32_t bf, int32_t n_error_buf,
                             int32_t max_box, int64_t ntag, const int32_t* tags, int32_t* boxes_out, int32_t cap,
                             int32_t* nboxes);
sh_status sh_local_nest_boxes(int32_t M_level, int32_t nadded, const int32_t* added_fine, int32_t nlevel,
                              const int32_t* level_boxes, int32_t bf, int32_t max_box, int32_t* boxes_out, int32_t cap,
                              int32_t* nboxes);

/* Wait for all work queued by this hierarchy; SH_EDEVICE if any kernel failed. */
sh_status sh_sync(sh_hierarchy h);

/* Release the handle and the library's index tables (after waiting for its queued
   work).  Caller-owned arenas are not touched and may be freed afterwards. */
sh_status sh_hierarchy_destroy(sh_hierarchy h);

/* Message of the last non-OK status returned on this thread (never NULL). */
const char* sh_last_error(void);

/* Rebind the hierarchy to another HIP stream (its later work is queued there).  The
   caller orders the switch: work still queued on the old stream must be complete or
   waited for before the new stream touches the hierarchy (e.g. set up on one stream,
   record an event, and join a batch on another once it has passed).  Used by the
   ensemble server to set jobs up beside the running batch. */
sh_status sh_set_stream(sh_hierarchy h, void* hip_stream);

/* Set every level's step counter back to 0 (time eta0), queued on the stream, so that
   a hierarchy can be reused for a new run of the same layout after sh_write_state of the
   new initial state and sh_fill_ghosts (the ensemble server reuses the hierarchies of
   finished jobs instead of allocating new ones).  Errors: SH_ESTATE (no levels, an active
   shadow level, while recording). */
sh_status sh_restart(sh_hierarchy h);

/* Debugging aid, not part of the level step (flags, 0 = off): bit 0 writes NaN into the
   ghost shell of a buffer (all its layers, the components the fill carries) just before
   every fill that is meant to set all of it (stage inputs between stages, U_n at the end
   of a level step, sh_fill_ghosts, tagging), so that a ghost cell some stencil reads but
   no fill writes turns valid cells into NaN instead of silently reusing stale values.
   Results are unchanged when every read ghost is filled.  Errors: SH_EINVAL (unknown
   flag), SH_ESTATE (while recording). */
sh_status sh_set_debug(sh_hierarchy h, int32_t flags);

/* Measurement support, not part of the level step: the HBM bandwidth a plain kernel
   reaches on this device, as the achievable ceiling beside the nominal peak.  One launch
   of `bytes` (a positive multiple of 16) with 16-byte nontemporal accesses, on
   `hip_stream`: kind 0 reads `src` (device; nothing is written to `dst`, which must
   still be a device buffer of at least 16 bytes), 1 writes `dst` (device), 2 copies src
   to dst (device, not overlapping).  Both pointers 16-byte aligned.  Queued; errors:
   SH_EINVAL (bad kind, size or alignment), SH_EDEVICE (launch failed). */
sh_status sh_stream_probe(int32_t kind, const void* src, void* dst, int64_t bytes, void* hip_stream);

/* Stage scalars the device derives for `lev` at stage s (0..3 for RK4, 0..2 for SSPRK3)
   of the current step: out[0..6] = {eta_s, c_fric, c_pot, dt/6, dt/3, dt/2, dt}.
   Diagnostic. */
sh_status sh_debug_stage_scalars(sh_hierarchy h, int32_t lev, int32_t s, double* out_host);

/* Launch shape (performance only; results are identical for every choice).
   kind: 0 = per-stage kernel with one wavefront per 64-cell tile for every box; 4 or 8 =
     blocks of that many wavefront rows sharing psi (and Pi under dissipation) through
     LDS for boxes at least 64 cells wide.
   nontemporal: 1 = once-used streams do not stay cache resident.
   tile_z: cells per per-stage tile in z (0 = from the level size: 64, halved down to 1
     while the level has fewer than 16384 tiles).
   fuse: 4 = level 0 (which has no coarse/fine boundary) takes each step in one kernel
     computing all the integrator's stages (temporal blocking; needs every level-0 box to
     be a multiple of the fused footprint, else per-stage); 0 = per-stage kernels.
   fused_shape: footprint 0 = 32 x 8, 1 = 64 x 4, 2 = 32 x 16, 3 = 16 x 8.
   fused_tile_z: planes per fused tile; 0 = 512, halved while that gives fewer than 1024
     tiles, down to 16 (a batch decides once for all its members).
   fused_variant: thread order / x-neighbour exchange / accumulator placement / U_n
     prefetch of the fused kernel: 0 = row-major, LDS, registers; 1 = row-major, lane
     shifts, registers; 2 = row-major, lane shifts, LDS; 3 = ring order, LDS, LDS; 4 =
     ring order, LDS, registers; 5 = as 4 with U_n planes loaded two iterations ahead; 6 =
     as 5 with the accumulator in LDS; 7 = as 3 with the U_n values of stages 1 and 2
     read again from memory instead of kept in registers; 8 = as 7 with the two-iteration
     prefetch (SSPRK3 has no accumulator: 2, 3 and 6 run as 1, 4 and 5).
   Applies to every level.  Defaults at creation: kind 8, nontemporal 1, tile_z 0, fuse 4,
   fused_tile_z 0, fused_shape 2 with fused_variant 3 for RK4 in SH_F64, 6 for RK4 in
   SH_F32 and 5 for SSPRK3.  The environment variable SHAMR_TUNE (e.g.
   "kind=8,nt=1,zc=0,fuse=4,fshape=0,fzc=0,fvar=5,fgrp=1") overrides them; fgrp 1 = fused
   tiles launched in groups of 32 covering square-ish patches, 0 = in rows. */
sh_status sh_set_tuning(sh_hierarchy h, int32_t kind, int32_t nontemporal, int32_t tile_z, int32_t fuse,
                        int32_t fused_shape, int32_t fused_tile_z, int32_t fused_variant);

/* Per-kernel timing (diagnostic).  sh_profile(h, 1) clears the totals and brackets every
   launch that sh_advance_level and sh_average_down issue with HIP events on the
   hierarchy's stream; sh_profile(h, 0) stops.  sh_profile_read fills ms[8] (summed
   event time) and counts[8] (launches) per class: 0-3 = RK stage 1-4 kernel, 4 =
   same-level ghost copy, 5 = coarse/fine ghost interpolation, 6 = average down,
   7 = fused four-stage step kernel.  Reading synchronises the stream. */
sh_status sh_profile(sh_hierarchy h, int32_t enable);
sh_status sh_profile_read(sh_hierarchy h, double* ms, int64_t* counts);

/* Batched stepping of independent simulations (ensemble serving).  A batch groups
   single-level hierarchies of one precision created on one stream; sh_batch_advance
   takes one RK4 step of every member with one launch per kernel (fused step, or the four
   stage kernels and their ghost copies, then the step counters and the ghost copy of the
   new states), so small lattices share the GPU instead of each filling it alone.  Each
   member's result is bit-identical to stepping it alone (kernels are gather-only per
   box).  Members must not be re-laid out or destroyed while the batch exists; the batch
   borrows them.  Errors: SH_EINVAL (a member with more than one level, another
   precision or stream, an integrator other than RK4, a Laplacian order other than 1 or
   dissipation),
   SH_ESTATE from sh_batch_advance if a member's layout changed
   since the batch was built. */
sh_status sh_batch_create(int32_t njobs, const sh_hierarchy* jobs, sh_batch* out);
/* Replace a batch's members (same rules as sh_batch_create) without releasing its device
   tables: the new tables are copied in stream order, so launches queued before the call
   still run on the old members, and the call waits for the stream only when a table
   outgrows its buffer.  Graphs recorded from the batch before the call must not be
   launched afterwards. */
sh_status sh_batch_update(sh_batch b, int32_t njobs, const sh_hierarchy* jobs);
sh_status sh_batch_advance(sh_batch b);
sh_status sh_batch_destroy(sh_batch b);

/* Truncation error estimates (Sec. II.B "self-shadow"; Sec. IV.C).  With sh_set_tee(h, 1,
   te_crit, tag_mode) every sh_average_down first computes, per coarse cell it covers,
   TEE = max over the four components of |C - avg(children)| (float64, the first
   component's value unless a later one compares greater) and stores it on the fine
   level's cells (all 8 children), before overwriting C.  Level 0 has no coarser level:
   sh_shadow_begin(h) (level 0 at an even step count, even-aligned level-0 boxes) builds
   the shadow level, level 0 averaged onto half its resolution; sh_shadow_advance(h)
   takes its single step of twice the level-0 step; once level 0 has taken its two steps,
   sh_shadow_end(h) stores the same estimate (shadow against level 0 averaged) on level
   0 and releases the shadow.  On a regrid kept cells keep their estimate and new cells
   start at 0.  tag_mode selects what sh_tag_cells tags: 1 = plaquette winding, 2 =
   estimate > te_crit, 3 = either.  sh_read_tee copies a level's estimates (one double
   per valid cell, boxes in layout order, x fastest) to device memory of the caller.
   Errors: SH_EINVAL (bad tag_mode or te_crit, odd or misaligned level 0), SH_ESTATE
   (shadow calls out of order). */
sh_status sh_set_tee(sh_hierarchy h, int32_t enable, double te_crit, int32_t tag_mode);
sh_status sh_shadow_begin(sh_hierarchy h);
sh_status sh_shadow_advance(sh_hierarchy h);
sh_status sh_shadow_end(sh_hierarchy h);
sh_status sh_read_tee(sh_hierarchy h, int32_t lev, double* out_dev);

/* Per-field estimates and their modifier (Sec. IV.C "Modifying truncation error
   estimates"; App. D), for a hierarchy created with tee_fields = 1: every synchronisation
   (and sh_shadow_end) keeps each component's own estimate D_c = |C_c - avg(children)_c|,
   and tagging by estimate marks a cell where f_c(D_c) > te_crit[c] for some component c,
   with the modifier f_c(D) = scale[c] * D (float64).  The paper's modifier is a user
   function; the one built here is the rescaling its App. D applies (D_phi / max phi and
   D_phi' / max phi'), with scale[c] supplied by the caller, e.g. 1 / sh_field_absmax.
   te_crit[4] and scale[4] (NULL = all 1) are host arrays, finite and >= 0; they apply at
   the next sh_tag_cells, so the scales can be renewed before each regrid without
   touching the estimates already formed.  sh_set_tee on such a hierarchy sets every
   threshold to te_crit and every scale to 1 (the same tags as one estimate per cell).
   sh_read_tee then writes 4 x (valid cells) doubles, component after component.
   Errors: SH_ESTATE (tee_fields = 0), SH_EINVAL (bad tag_mode, threshold or scale). */
sh_status sh_set_tee_fields(sh_hierarchy h, int32_t enable, const double* te_crit, const double* scale,
                            int32_t tag_mode);

/* out_host[c] = max |U_c| over the valid cells of every level (c = psi1, psi2, Pi1, Pi2;
   NaN if any value is NaN): the field maxima App. D normalises the estimates by.
   Synchronises. */
sh_status sh_field_absmax(sh_hierarchy h, double* out_host);

/* Recorded level steps (HIP graphs).  The Berger-Oliger order of Sec. II.A (Fig. 2) is a
   fixed sequence of launches for a fixed layout, so a coarse step (or several) can be
   recorded once and replayed with one launch; the step counters and level times live in
   device memory, so every replay advances the simulation.
   sh_capture_begin(h) starts recording on h's stream: until sh_capture_end, the calls
   sh_advance_level, sh_average_down and sh_fill_ghosts are recorded, not run; every
   call that synchronises, allocates, uploads or reads back (layout, state I/O, tagging,
   energy, sync, tuning, profiling, tracing) fails with SH_ESTATE.  Profiling and tracing
   must be off.  sh_capture_end(h, &g) stops recording and returns the graph; the host
   step counters are as before the capture.  sh_batch_capture(b, nsteps, &g) records
   nsteps batch steps.  sh_graph_launch(g) replays on the recording stream (asynchronous)
   and advances the host step counters by what was recorded; SH_ESTATE if a recorded
   hierarchy's layout changed since.  sh_graph_destroy releases it (the caller owns g;
   destroy graphs before the hierarchies they record). */
sh_status sh_capture_begin(sh_hierarchy h);
sh_status sh_capture_end(sh_hierarchy h, sh_graph* out);
sh_status sh_batch_capture(sh_batch b, int32_t nsteps, sh_graph* out);
sh_status sh_graph_launch(sh_graph g);
sh_status sh_graph_destroy(sh_graph g);

/* Orchestration trace (diagnostic).  sh_trace(h, 1) clears and starts recording every
   operation that sh_advance_level and sh_average_down issue, as 4 int32 each
   (op, level, a, b): op 1 = RK stage a (0..3) of substep b; op 2 = same-level ghost copy
   of role a; op 3 = coarse/fine ghost interpolation of role a at alpha_num b; op 4 =
   average down of level `level` onto level-1.  sh_trace(h, 0) stops.  sh_trace_read
   copies up to `cap` records to `out` and returns the number recorded. */
sh_status sh_trace(sh_hierarchy h, int32_t enable);
int64_t sh_trace_read(sh_hierarchy h, int32_t* out, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif /* SHAMR_H */
