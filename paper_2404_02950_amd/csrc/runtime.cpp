// Host runtime of libshamr: hierarchy, box layouts, copy/interpolation/averaging plans,
// the level step sequence and the C-ABI declared in include/shamr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "shamr.h"
#include "sh_geom.h"
#include "sh_internal.h"
#include "sh_launch.h"

static thread_local std::string g_err;

static sh_status fail(sh_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(SH_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

#define LAUNCHCHK()                                                                    \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess) return fail(SH_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------------
// Device arrays for index tables (allocated at layout time only).
// ---------------------------------------------------------------------------------
// During a layout change the table uploads are staged in a pinned host buffer of the
// hierarchy and queued on its stream instead of one synchronous copy each (a layout change
// uploads a score of tables); the change synchronises the stream before the buffer is
// used again.  Outside a layout change (no stage set on this thread) uploads are
// synchronous.
struct UploadStage {
  hipStream_t st = nullptr;
  char* buf = nullptr;  // pinned (hipHostMalloc)
  size_t cap = 0, used = 0, want = 0;
  bool queued = false;
};
thread_local UploadStage* g_stage = nullptr;

template <typename T>
struct DevArr {
  T* p = nullptr;
  size_t n = 0;
  hipError_t upload(const std::vector<T>& v) {
    release();
    n = v.size();
    if (n == 0) return hipSuccess;
    const size_t bytes = n * sizeof(T);
    hipError_t e = hipMalloc((void**)&p, bytes);
    if (e != hipSuccess) { p = nullptr; n = 0; return e; }
    UploadStage* sg = g_stage;
    if (sg) {
      sg->want += (bytes + 255) / 256 * 256;
      if (sg->buf && sg->used + bytes <= sg->cap) {
        char* h = sg->buf + sg->used;
        std::memcpy(h, v.data(), bytes);
        sg->used += (bytes + 255) / 256 * 256;
        sg->queued = true;
        return hipMemcpyAsync(p, h, bytes, hipMemcpyHostToDevice, sg->st);
      }
    }
    return hipMemcpy(p, v.data(), bytes, hipMemcpyHostToDevice);
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// Segments and their work chunks: chunk k covers cells [start, start + CHUNK) of one
// segment (one workgroup per chunk, or one wavefront for CHUNK = SH_WAVE).
template <typename S, int CHUNK = SH_BLOCK>
struct SegPlan {
  DevArr<S> segs;
  DevArr<SegBlock> blocks;
  long long ncells = 0;
  int nblocks() const { return (int)blocks.n; }
  hipError_t upload(const std::vector<S>& v, const std::vector<long long>& ncell_per_seg) {
    std::vector<SegBlock> b;
    ncells = 0;
    for (size_t i = 0; i < v.size(); ++i) {
      for (long long s = 0; s < ncell_per_seg[i]; s += CHUNK) b.push_back(SegBlock{(int)i, (int)s});
      ncells += ncell_per_seg[i];
    }
    hipError_t e = segs.upload(v);
    if (e != hipSuccess) return e;
    return blocks.upload(b);
  }
  void release() {
    segs.release();
    blocks.release();
    ncells = 0;
  }
};

// ---------------------------------------------------------------------------------
// Level layout arithmetic (shared by sh_arena_bytes and sh_set_level_layout).
// ---------------------------------------------------------------------------------
// Ghost layers of level 0 (enough for four fused RK stages); refined levels keep one.
#define SH_NG0 4

struct LayoutGeom {
  int ng = 1;                       // ghost layers
  int tee_nc = 1;                   // truncation error estimates per valid cell (1 or 4)
  int esize;                        // bytes of a stored value (8 or 4)
  int xoff;                         // elements before x = 0 in a row (x = 0 on 64 or 128 B)
  std::vector<long long> box_off;   // element offset of each box block
  std::vector<int> px;              // per-box x pitch
  std::vector<long long> cs;        // per-box component stride
  long long E = 0;                  // elements per slot
  long long nvalid = 0;
  std::vector<Tile> tiles;
  // arena byte offsets
  size_t off_slot[3], off_acc, off_mask, off_cov, off_cnt, off_toff, off_part, off_eout, off_tee, total;
};

static long long round_up(long long v, long long a) { return (v + a - 1) / a * a; }

// Planes per tile: 64, halved (down to zmin) while the level would have fewer than 16384
// wave tiles.  The per-stage kernels of small refined levels run fastest with single-plane
// tiles (more wavefronts in flight outweigh the z-window reuse); tagging and energy tiles
// keep at least 4.
static int tile_zc_default(long long cells, int zmin = 4) {
  const char* env = std::getenv("SHAMR_TILE_Z");
  if (env) {
    int v = std::atoi(env);
    if (v >= 1 && v <= 1024) return v;
  }
  long long zc = 64;
  while (zc > zmin && cells / (64LL * zc) < 16384) zc >>= 1;
  return (int)zc;
}

// Stages per step of the integrator: 4 for classic RK4 (types 0 and 4), 3 for SSPRK3
// (types 3 and 10) and RKN4 (type 21).
// (types 3 and 10).  SSPRK3 keeps no accumulator, so its levels store three states per
// cell instead of three plus a float64 accumulator.
static int stages_of(const sh_params& p) {
  return (p.integrator == 3 || p.integrator == 10 || p.integrator == 21) ? 3 : 4;
}
// RKN4 (integrator type 21): three stages in the role cycle of the three-stage methods,
// with a float64 accumulator like RK4's.  RKN5 (type 22): four stages over three slots in
// a cycle of its own (role_slot), the float64 accumulator holding the position and
// velocity sums; single periodic levels only.
static bool rkn5_of(const sh_params& p) { return p.integrator == 22; }
static bool rkn_of(const sh_params& p) { return p.integrator == 21 || rkn5_of(p); }
static bool needs_acc(const sh_params& p) { return stages_of(p) == 4 || rkn_of(p); }
// device stage id of stage s (0-based): RK4 0..3, SSPRK3 4..6, RKN4 7..9, RKN5 10..13
static int stage_id(const sh_params& p, int s) {
  return rkn5_of(p) ? 10 + s : (p.integrator == 21 ? 7 + s : (stages_of(p) == 3 ? 4 + s : s));
}
// slot-cycle code kept with the level scalars: the stage count, or 5 for RKN5
static int slot_cycle(const sh_params& p) { return rkn5_of(p) ? 5 : stages_of(p); }

// Laplacian order of appendix A (1, 2, 3: the 7-, 13-, 19-point stencil; 0 reads as 1).
// Refined levels (and the shadow level) keep a ghost shell of that depth; level 0 keeps
// SH_NG0 >= 3 for the fused step.
static int lap_order_of(const sh_params& p) { return p.lap_order > 1 ? p.lap_order : 1; }

// Spatial interpolation of appendix E: 1 = linear conservative (0 reads as 1), 4 = quartic
// conservative.  Its coarse support reaches 1 or 2 coarse cells beyond the parent, so with
// quartic interpolation refined levels keep at least two ghost layers (a level is the
// coarse level of the next one).
static int interp_of(const sh_params& p) { return p.interp == 4 ? 4 : 1; }
static int interp_reach(const sh_params& p) { return interp_of(p) == 4 ? 2 : 1; }

// Kreiss-Oliger dissipation order (0 = off, 2, 3 = the ghost cells its stencil needs).  It
// stencils Pi as well as psi, so the fills between stages then carry all four
// components (and the block-row stage kernel stages Pi through LDS as well).
static int ko_of(const sh_params& p) { return p.ko_order; }
static double ko_coef(const sh_params& p, double dx) {
  if (p.ko_order == 2) return -p.ko_eps / (16.0 * dx);
  if (p.ko_order == 3) return p.ko_eps / (64.0 * dx);
  return 0.0;
}
// ghost cells a stage reads, and components the fills between stages carry
static int stencil_depth(const sh_params& p) { return std::max(lap_order_of(p), ko_of(p)); }
static int fill_comps(const sh_params& p) { return ko_of(p) ? 4 : 2; }
static int refined_ng(const sh_params& p) { return std::max(stencil_depth(p), interp_reach(p)); }
// truncation error estimates kept per cell: one per component when asked for, else their maximum
static int tee_comps(const sh_params& p) { return p.tee_fields ? 4 : 1; }
// the fused level-0 step: 7-point stencil, no dissipation
static bool fusable(const sh_params& p) { return lap_order_of(p) == 1 && ko_of(p) == 0 && !rkn_of(p); }

static void make_geom(int prec, int ng, const std::vector<IBox>& boxes, LayoutGeom& g, bool acc, int tee_nc = 1) {
  g.ng = ng;
  g.tee_nc = tee_nc;
  g.esize = prec == SH_F64 ? 8 : 4;
  // x = 0 starts a 128-byte line for float64 where the ghost shell is thin (refined and
  // shadow levels: narrow rows of 8-64 cells then fill whole lines), 64 bytes in
  // otherwise (level 0's shell of 4, whose x-ghost runs the copy plan widens to whole
  // sectors; float32 rows, which a 128-byte start only makes longer)
  g.xoff = (ng < SH_NG0 && g.esize == 8 ? 128 : 64) / g.esize;
  g.box_off.clear();
  g.px.clear();
  g.cs.clear();
  g.tiles.clear();
  g.E = 0;
  g.nvalid = 0;
  for (const IBox& b : boxes) {
    const int nx = b.size(0), ny = b.size(1), nz = b.size(2);
    const int px = (int)round_up(g.xoff + nx + ng, g.xoff);
    const long long cs = round_up((long long)px * (ny + 2 * ng) * (nz + 2 * ng), 64);
    g.box_off.push_back(g.E);
    g.px.push_back(px);
    g.cs.push_back(cs);
    g.E += 4 * cs;
    g.nvalid += (long long)nx * ny * nz;
  }
  const int zc = tile_zc_default(g.nvalid);
  for (size_t bi = 0; bi < boxes.size(); ++bi) {
    const IBox& b = boxes[bi];
    const int nx = b.size(0), ny = b.size(1), nz = b.size(2);
    int txs = 0;
    while ((1 << txs) < nx && txs < 6) ++txs;
    const int TX = 1 << txs, TY = 64 / TX;
    for (int z0 = 0; z0 < nz; z0 += zc)
      for (int y0 = 0; y0 < ny; y0 += TY)
        for (int x0 = 0; x0 < nx; x0 += TX) {
          Tile t;
          t.box = (int)bi;
          t.xy = x0 | (y0 << 16);
          t.zz = z0 | (std::min(zc, nz - z0) << 16);
          t.txs = txs;
          g.tiles.push_back(t);
        }
  }
  const long long nt = (long long)g.tiles.size();
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = (size_t)round_up((long long)(o + bytes), 256);
    return r;
  };
  for (int s = 0; s < 3; ++s) g.off_slot[s] = take((size_t)g.E * g.esize);
  g.off_acc = acc ? take((size_t)g.E * 8) : 0;
  g.off_mask = take((size_t)g.nvalid);
  g.off_cov = take((size_t)g.nvalid);
  g.off_cnt = take((size_t)nt * 4);
  g.off_toff = take((size_t)(nt + 1) * 8);
  g.off_part = take((size_t)nt * sizeof(EnergyPartial));
  g.off_eout = take(4 * 8);
  g.off_tee = take((size_t)g.nvalid * 8 * g.tee_nc);  // truncation error estimates per valid cell
  g.total = o + 256;  // slack for aligning the arena base
}

// Stage-kernel launch shape.  kind: 0 = wave-row tiles for every box; 4 or 8 = block
// rows of that many wavefronts for boxes at least 64 cells wide (narrower boxes keep
// wave-row tiles).  nt: nontemporal once-used streams.  zc: cells per tile in z (0 =
// chosen from the level size).
// fuse: 4 = level 0 advances with the fused kernel (all stages of a step in one launch)
// when its boxes are multiples of the fused footprint (fshape 0: 32 x 8, 1: 64 x 4, 2: 32 x 16, 3: 16 x 8), 0 =
// per-stage kernels.
struct Tuning {
  int kind = 8;
  int nt = 1;
  int zc = 0;
  int fuse = 4;
  int fshape = 0;
  int fzc = 0;   // planes per fused tile; 0 = chosen from the number of tiles
  int fvar = 0;  // fused kernel variant (thread order / neighbour exchange / accumulator)
  int fgrp = 1;  // fused tile order: 1 = groups of 32 tiles on square-ish patches, 0 = rows
};

// Fastest fused launches measured at 512^3 on MI355X, all on the 32 x 16 footprint (15
// wavefronts per workgroup, so at most 128 registers): RK4 FP64 variant 3 (accumulator in
// LDS, ring-ordered threads; 3.11 ms against 3.23 ms for variant 7), RK4 FP32 variant 6
// (1.92 ms); SSPRK3 variant 5 in both precisions (2.18 and 1.36 ms).
static Tuning default_tuning(const sh_params& p) {
  Tuning t;
  t.fshape = 2;
  if (stages_of(p) == 3) {
    t.fvar = 5;
  } else if (p.prec == SH_F32) {
    t.fvar = 6;
  } else {
    t.fvar = 3;
  }
  return t;
}

static void tuning_from_env(Tuning& t) {
  const char* env = std::getenv("SHAMR_TUNE");  // e.g. "kind=8,nt=1,zc=32"
  if (!env) return;
  std::string s(env);
  size_t pos = 0;
  while (pos < s.size()) {
    size_t end = s.find(',', pos);
    if (end == std::string::npos) end = s.size();
    const std::string kv = s.substr(pos, end - pos);
    const size_t eq = kv.find('=');
    if (eq != std::string::npos) {
      const std::string k = kv.substr(0, eq);
      const int v = std::atoi(kv.c_str() + eq + 1);
      if (k == "kind" && (v == 0 || v == 4 || v == 8)) t.kind = v;
      if (k == "nt" && (v == 0 || v == 1)) t.nt = v;
      if (k == "zc" && v >= 0 && v <= 1024) t.zc = v;
      if (k == "fuse" && (v == 0 || v == 4)) t.fuse = v;
      if (k == "fshape" && v >= 0 && v <= 3) t.fshape = v;
      if (k == "fzc" && v >= 0 && v <= 1024) t.fzc = v;
      if (k == "fvar" && v >= 0 && v <= 8) t.fvar = v;
      if (k == "fgrp" && (v == 0 || v == 1)) t.fgrp = v;
    }
    pos = end + 1;
  }
}

static void make_stage_tiles(const std::vector<IBox>& boxes, const Tuning& tu, long long nvalid,
                             std::vector<Tile>& wt, std::vector<Tile>& bt) {
  wt.clear();
  bt.clear();
  int zc = tu.zc > 0 ? tu.zc : tile_zc_default(nvalid, 1);
  for (size_t bi = 0; bi < boxes.size(); ++bi) {
    const IBox& b = boxes[bi];
    const int nx = b.size(0), ny = b.size(1), nz = b.size(2);
    if (tu.kind != 0 && nx >= 64) {
      const int R = tu.kind;
      for (int z0 = 0; z0 < nz; z0 += zc)
        for (int y0 = 0; y0 < ny; y0 += R)
          for (int x0 = 0; x0 < nx; x0 += 64) {
            Tile t;
            t.box = (int)bi;
            t.xy = x0 | (y0 << 16);
            t.zz = z0 | (std::min(zc, nz - z0) << 16);
            t.txs = 6;
            bt.push_back(t);
          }
      continue;
    }
    int txs = 0;
    while ((1 << txs) < nx && txs < 6) ++txs;
    const int TX = 1 << txs, TY = 64 / TX;
    for (int z0 = 0; z0 < nz; z0 += zc)
      for (int y0 = 0; y0 < ny; y0 += TY)
        for (int x0 = 0; x0 < nx; x0 += TX) {
          Tile t;
          t.box = (int)bi;
          t.xy = x0 | (y0 << 16);
          t.zz = z0 | (std::min(zc, nz - z0) << 16);
          t.txs = txs;
          wt.push_back(t);
        }
  }
}

// Tiles of the fused step; empty if some box is not a multiple of the footprint.
// Fused tiles in launch order.  Blocks go round-robin to the 8 XCDs and the kernel maps
// each XCD to one contiguous run of the tile list, whose first 32 entries (one per CU)
// then run together.  Listing the tiles of a box by groups of 32 that cover a square-ish
// patch (not a strip of whole rows) lets those concurrent tiles share most of their
// halo columns in the XCD's L2.
// Whether a level's boxes can take the fused step, and how many footprint columns they
// have in total.
static long long fused_columns(const std::vector<IBox>& boxes, const Tuning& tu, int ng) {
  if (tu.fuse != 4 || ng < 4) return 0;
  int TX, TY;
  sh_fused_footprint(tu.fshape, &TX, &TY);
  long long n = 0;
  for (const IBox& b : boxes) {
    if (b.size(0) % TX || b.size(1) % TY) return 0;
    n += (long long)(b.size(0) / TX) * (b.size(1) / TY);
  }
  return n;
}

// Planes per fused tile when not set: long columns (each tile re-reads and recomputes
// 2 * FG planes at its ends) unless that leaves fewer than 4 tiles per CU, then shorter
// ones down to 16 planes (small lattices would otherwise run on a few CUs).
static int fused_zc(const Tuning& tu, long long columns, int nz_max) {
  if (tu.fzc > 0) return tu.fzc;
  int zc = 512;
  while (zc > 16 && columns * ((nz_max + zc - 1) / zc) < 1024) zc >>= 1;
  return zc;
}

static void make_fused_tiles(const std::vector<IBox>& boxes, const Tuning& tu, int ng, std::vector<Tile>& ft,
                             int zc_given = 0) {
  ft.clear();
  const long long columns = fused_columns(boxes, tu, ng);
  if (columns == 0) return;
  int TX, TY;
  sh_fused_footprint(tu.fshape, &TX, &TY);
  int nz_max = 1;
  for (const IBox& b : boxes) nz_max = std::max(nz_max, b.size(2));
  const int fzc = zc_given > 0 ? zc_given : fused_zc(tu, columns, nz_max);
  // group of GX x GY tiles with GX * GY = 32 and GX * TX close to GY * TY
  int GX = 1;
  while (GX < 32 && (long long)(2 * GX) * TX <= (long long)(32 / (2 * GX)) * TY * 2) GX *= 2;
  int GY = 32 / GX;
  if (!tu.fgrp) {
    GX = 1 << 30;
    GY = 1;
  }
  for (size_t bi = 0; bi < boxes.size(); ++bi) {
    const IBox& b = boxes[bi];
    const int nx = b.size(0), ny = b.size(1), nz = b.size(2);
    const int ntx = nx / TX, nty = ny / TY;
    for (int z0 = 0; z0 < nz; z0 += fzc)
      for (int gy = 0; gy < nty; gy += GY)
        for (int gx = 0; gx < ntx; gx += GX)
          for (int ty = gy; ty < std::min(gy + GY, nty); ++ty)
            for (int tx = gx; tx < std::min(gx + GX, ntx); ++tx) {
              Tile t;
              t.box = (int)bi;
              t.xy = (tx * TX) | ((ty * TY) << 16);
              t.zz = z0 | (std::min(fzc, nz - z0) << 16);
              t.txs = tu.fshape;
              ft.push_back(t);
            }
  }
}

// ---------------------------------------------------------------------------------
// Hierarchy
// ---------------------------------------------------------------------------------
struct Level {
  int M = 0;
  double dx = 0, dt = 0;
  std::vector<IBox> boxes;
  LayoutGeom g;
  char* base = nullptr;  // aligned arena base
  std::vector<BoxDev> hbox;
  DevArr<BoxDev> dbox;
  DevArr<Tile> tiles;             // wave tiles of every box (tagging, energy, rhs)
  DevArr<Tile> stiles_w, stiles_b;  // stage-kernel tiles: wave rows / block rows
  DevArr<long long> xoff_valid, xoff_ghost, rhs_off;
  SegPlan<CopySeg, SH_WAVE> a1;    // same-level ghost copy, one layer (a wavefront per chunk)
  SegPlan<CopySeg, SH_WAVE> a1d;   // the same over the whole ghost depth (when deeper than one)
  DevArr<Tile> ftiles;    // fused-step tiles (level 0 only)
  SegPlan<InterpSeg> a2;  // coarse -> this level's ghosts
  SegPlan<AvgSeg> a5;     // this level -> coarse level
  long long k = 0;        // host mirror of the device step counter
  bool stale = false;     // coarse level changed; layout must be set again
  int* d_idx = nullptr;   // tag compaction output (grown on demand)
  long long d_idx_cap = 0;
  BoxBins bins;

  uint8_t* mask() const { return (uint8_t*)(base + g.off_mask); }
  uint8_t* covered() const { return (uint8_t*)(base + g.off_cov); }
  double* tee() const { return (double*)(base + g.off_tee); }
  int* tile_count() const { return (int*)(base + g.off_cnt); }
  long long* tile_off() const { return (long long*)(base + g.off_toff); }
  EnergyPartial* epart() const { return (EnergyPartial*)(base + g.off_part); }
  double* eout() const { return (double*)(base + g.off_eout); }
  int ntiles() const { return (int)g.tiles.size(); }

  void release_tables() {
    dbox.release();
    tiles.release();
    stiles_w.release();
    stiles_b.release();
    xoff_valid.release();
    xoff_ghost.release();
    rhs_off.release();
    a1.release();
    a1d.release();
    ftiles.release();
    a2.release();
    a5.release();
  }
  void release() {
    release_tables();
    if (d_idx) (void)hipFree(d_idx);
    d_idx = nullptr;
    d_idx_cap = 0;
  }
};

struct sh_hierarchy_s {
  sh_params p;
  Tuning tune;
  hipStream_t st = nullptr;
  int dev = 0;  // the HIP device current at creation (its arenas and stream are on it)
  // graph capture: while capturing, level steps are recorded, not run; the host step
  // counters are put back at the end and advanced by each replay instead
  bool capturing = false;
  std::vector<long long> k_at_capture;
  // truncation error estimates (computed at every synchronisation when on) and the
  // tagging criterion: bit 0 plaquette winding, bit 1 estimate above its threshold
  // (te.crit[0] for one estimate per cell; te.scale[c] * estimate_c > te.crit[c] per field)
  int debug = 0;  // bit 0: NaN into ghost shells before every complete fill
  bool tee_on = false;
  TeeSpec te = {{0.0, 0.0, 0.0, 0.0}, {1.0, 1.0, 1.0, 1.0}, 1, 0};
  int tag_mode = 1;
  // shadow level: level 0 averaged onto half its resolution, evolved by one step of
  // twice the level-0 step (its scalars live in d_ls[SH_SHADOW_LS]; arena owned here)
  bool has_shadow = false;
  Level shadow;
  char* shadow_arena = nullptr;
  long long shadow_k0 = 0;
  SegPlan<AvgSeg> shadow_a5;
  long long layout_version = 0;  // bumped by every layout change (captured graphs go stale)
  LevelScal* d_ls = nullptr;  // 16 levels, then the shadow level
  UploadStage stage;          // pinned staging of the table uploads of a layout change
  // octant bitsets of tagged blocks (sh_tag_blocks): device buffer of 8 x oct_words words
  // and its host copy
  unsigned long long* d_oct = nullptr;
  long long oct_words = 0;
  std::vector<uint64_t> h_oct;
  double* d_dbg = nullptr;
  std::vector<Level> lev;
  bool tracing = false;
  std::vector<int32_t> trace;  // (op, level, a, b) records
  // per-kernel-class event timing: pairs of events around launches
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_class;  // class of each recorded pair
  double prof_ms[8] = {0};
  long long prof_n[8] = {0};
  hipEvent_t prof_begin() {
    if (!profiling) return nullptr;
    if (ev_used + 2 > ev_pool.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ev_pool.push_back(e);
      }
    }
    hipEvent_t e = ev_pool[ev_used];
    (void)hipEventRecord(e, st);
    return e;
  }
  void prof_end(hipEvent_t b, int cls) {
    if (!profiling || !b) return;
    (void)hipEventRecord(ev_pool[ev_used + 1], st);
    ev_used += 2;
    ev_class.push_back(cls);
  }
  void prof_collect() {
    if (ev_used == 0) return;
    (void)hipStreamSynchronize(st);
    for (size_t i = 0; i < ev_class.size(); ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev_pool[2 * i], ev_pool[2 * i + 1]) == hipSuccess) {
        prof_ms[ev_class[i]] += ms;
        prof_n[ev_class[i]] += 1;
      }
    }
    ev_used = 0;
    ev_class.clear();
  }
  void rec(int op, int l, int a, int b) {
    if (!tracing) return;
    trace.push_back(op);
    trace.push_back(l);
    trace.push_back(a);
    trace.push_back(b);
  }
};

constexpr int SH_SHADOW_LS = 16;  // slot of the shadow level's scalars in d_ls (after 16 levels)

static double level_dx(const sh_params& p, int l) { return (p.L / (double)p.n0) / (double)(1 << l); }

static LevelScal make_ls(const sh_params& p, int l, long long k) {
  LevelScal s;
  s.dx = level_dx(p, l);
  s.dt = p.cfl * s.dx;
  s.eta0 = p.eta0;
  s.alpha = p.alpha_fric;
  s.lam = p.lambda;
  s.inv_dx2 = 1.0 / (s.dx * s.dx);
  s.ko = ko_coef(p, s.dx);
  s.beta = p.beta_pot;
  s.nst = slot_cycle(p);
  s.k = k;
  return s;
}

static sh_status upload_ls(sh_hierarchy h, int l) {
  LevelScal s = make_ls(h->p, l, h->lev[l].k);
  HIPCHK(hipMemcpyAsync(h->d_ls + l, &s, sizeof(s), hipMemcpyHostToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return SH_OK;
}

static sh_status parse_boxes(const sh_params& p, int l, int nboxes, const int32_t* in, std::vector<IBox>& out) {
  out.clear();
  if (nboxes < 0 || (nboxes > 0 && !in)) return fail(SH_EINVAL, "bad box array");
  const int M = p.n0 << l;
  for (int i = 0; i < nboxes; ++i) {
    IBox b;
    for (int d = 0; d < 3; ++d) {
      b.lo[d] = in[6 * i + d];
      b.hi[d] = in[6 * i + 3 + d];
      if (b.lo[d] < 0 || b.hi[d] >= M || b.lo[d] > b.hi[d])
        return fail(SH_EINVAL, "box " + std::to_string(i) + " outside the level domain");
      if (b.size(d) > 32767) return fail(SH_EINVAL, "box side too large");
      if (l > 0 && ((b.lo[d] & 1) || !(b.hi[d] & 1)))
        return fail(SH_EINVAL, "box " + std::to_string(i) + " of a refined level must start even and end odd");
    }
    out.push_back(b);
  }
  // disjointness
  BoxBins bins;
  bins.build(out, M);
  for (int i = 0; i < nboxes; ++i) {
    bool bad = false;
    bins.query(out[i], [&](int j) {
      if (j != i && !isect(out[i], out[j]).empty()) bad = true;
    });
    if (bad) return fail(SH_EINVAL, "boxes overlap");
  }
  return SH_OK;
}

// ---------------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------------
static void build_a1(const Level& L, int depth, std::vector<CopySeg>& segs, std::vector<long long>& nc) {
  segs.clear();
  nc.clear();
  for (int d = 0; d < (int)L.boxes.size(); ++d) {
    const IBox& D = L.boxes[d];
    const IBox G = grow(D, depth);
    for_images(G, L.M, L.bins, [&](int s, const int sh[3]) {
      if (s == d && sh[0] == 0 && sh[1] == 0 && sh[2] == 0) return;
      const IBox img = shift(L.boxes[s], sh[0] * L.M, sh[1] * L.M, sh[2] * L.M);
      const IBox R = isect(G, img);
      if (R.empty()) return;
      CopySeg c;
      c.dbox = d;
      c.sbox = s;
      for (int k = 0; k < 3; ++k) {
        c.dlo[k] = R.lo[k] - D.lo[k];
        c.slo[k] = R.lo[k] - img.lo[k];
        c.n[k] = R.size(k);
      }
      c.pad = 0;
      segs.push_back(c);
      nc.push_back(R.volume());
    });
  }
  // One box spanning the periodic domain: its x-ghost runs are `depth` cells wide, a part
  // of one 64-byte memory sector on each side.  Widening them to the whole sector (the
  // x-padding before x = 0 and after the shell, which nothing reads) turns the partial
  // sector reads and writes of these runs into whole ones; the extra cells copy valid
  // cells.  Needs nx a multiple of the sector's element count and that much row padding.
  // Done for float64 only: in float32 a sector holds 16 cells and the wider runs measured
  // slower.
  if (L.boxes.size() == 1 && L.g.esize == 8) {
    const int xo = L.g.xoff, nx = L.boxes[0].size(0);
    if (L.boxes[0].size(0) == L.M && nx % xo == 0 && nx >= xo && L.g.px[0] >= 2 * xo + nx && depth <= xo) {
      for (size_t i = 0; i < segs.size(); ++i) {
        CopySeg& c = segs[i];
        if (c.n[0] != depth) continue;
        if (c.dlo[0] == -depth) {
          c.dlo[0] = -xo;
          c.slo[0] -= xo - depth;
        } else if (c.dlo[0] != nx) {
          continue;
        }
        c.n[0] = xo;
        nc[i] = (long long)c.n[0] * c.n[1] * c.n[2];
      }
    }
  }
}

// Host threads for the plan of a level with n boxes: one per 64 boxes, at most 8.
static int plan_workers(int n) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  return std::max(1, std::min({8, hw, n / 64}));
}

// Parents of fine region R (fine-global coordinates, possibly a ghost shell outside the
// domain) among the coarse boxes; appends InterpSegs for fine box d.  Returns false if
// some cell (or the one-cell slope support of its parent) is not covered.
static bool interp_segs(const Level& F, const Level& C, int d, const IBox& R, int reach, std::vector<InterpSeg>& segs,
                        std::vector<long long>& nc) {
  const IBox Pc = coarsen(R);
  long long covered = 0;
  for_images(Pc, C.M, C.bins, [&](int c, const int sh[3]) {
    const IBox img = shift(C.boxes[c], sh[0] * C.M, sh[1] * C.M, sh[2] * C.M);
    const IBox Q = isect(Pc, img);
    if (Q.empty()) return;
    const IBox sub = isect(R, refine(Q));
    if (sub.empty()) return;
    InterpSeg s;
    s.fbox = d;
    s.cbox = c;
    for (int k = 0; k < 3; ++k) {
      s.flo[k] = sub.lo[k] - F.boxes[d].lo[k];
      s.n[k] = sub.size(k);
      s.fg0[k] = sub.lo[k];
      s.cshift[k] = -img.lo[k];
    }
    segs.push_back(s);
    {
      // the plan counts tiles of parent cells (one SH_BLOCK-sized slot each)
      int np[3], qt[3];
      for (int k = 0; k < 3; ++k) np[k] = (sub.hi[k] >> 1) - (sub.lo[k] >> 1) + 1;
      qtile_dims(np, qt);
      long long nt = 1;
      for (int k = 0; k < 3; ++k) nt *= (np[k] + qt[k] - 1) / qt[k];
      nc.push_back(nt * SH_BLOCK);
    }
    covered += sub.volume();
  });
  if (covered != R.volume()) return false;
  const IBox sup = grow(Pc, reach);
  return covered_volume(sup, C.M, C.bins, C.boxes) == sup.volume();
}

// Coarse/fine ghost cells of F to a depth of `depth` cells (the stencil's reach; deeper
// ghost layers are only ever read as same-level copies), interpolated with coarse support
// `reach` cells around each parent.
// Boxes [b0, b1) of F; the plan is the concatenation over boxes in order.
static bool build_a2_range(const Level& F, const Level& C, int depth, int reach, int b0, int b1,
                           std::vector<InterpSeg>& segs, std::vector<long long>& nc) {
  std::vector<IBox> shell, rem, nxt;
  for (int d = b0; d < b1; ++d) {
    const IBox& D = F.boxes[d];
    shell.clear();
    subtract(grow(D, depth), D, shell);
    for (const IBox& P : shell) {
      rem.assign(1, P);
      for_images(P, F.M, F.bins, [&](int s, const int sh[3]) {
        const IBox img = shift(F.boxes[s], sh[0] * F.M, sh[1] * F.M, sh[2] * F.M);
        if (rem.empty() || isect(P, img).empty()) return;  // leaves rem as it is
        nxt.clear();
        for (const IBox& r : rem) subtract(r, img, nxt);
        rem.swap(nxt);
      });
      for (const IBox& R : rem)
        if (!interp_segs(F, C, d, R, reach, segs, nc)) return false;
    }
  }
  return true;
}

static bool build_a2(const Level& F, const Level& C, int depth, int reach, std::vector<InterpSeg>& segs,
                     std::vector<long long>& nc) {
  segs.clear();
  nc.clear();
  const int n = (int)F.boxes.size();
  const int nw = plan_workers(n);
  if (nw == 1) return build_a2_range(F, C, depth, reach, 0, n, segs, nc);
  std::vector<std::vector<InterpSeg>> ps(nw);
  std::vector<std::vector<long long>> pn(nw);
  std::vector<char> ok(nw, 0);
  std::vector<std::thread> th;
  for (int w = 0; w < nw; ++w)
    th.emplace_back([&, w] {
      ok[w] = build_a2_range(F, C, depth, reach, (int)((long long)n * w / nw), (int)((long long)n * (w + 1) / nw),
                             ps[w], pn[w]);
    });
  for (auto& t : th) t.join();
  for (int w = 0; w < nw; ++w) {
    if (!ok[w]) return false;
    segs.insert(segs.end(), ps[w].begin(), ps[w].end());
    nc.insert(nc.end(), pn[w].begin(), pn[w].end());
  }
  return true;
}

static bool build_a5(const Level& F, const Level& C, std::vector<AvgSeg>& segs, std::vector<long long>& nc) {
  segs.clear();
  nc.clear();
  for (int d = 0; d < (int)F.boxes.size(); ++d) {
    const IBox& D = F.boxes[d];
    const IBox Pc = coarsen(D);
    long long covered = 0;
    C.bins.query(Pc, [&](int c) {
      const IBox Q = isect(Pc, C.boxes[c]);
      if (Q.empty()) return;
      AvgSeg s;
      s.cbox = c;
      s.fbox = d;
      for (int k = 0; k < 3; ++k) {
        s.clo[k] = Q.lo[k] - C.boxes[c].lo[k];
        s.n[k] = Q.size(k);
        s.f0[k] = 2 * Q.lo[k] - D.lo[k];
      }
      s.pad = 0;
      segs.push_back(s);
      nc.push_back(Q.volume());
      covered += Q.volume();
    });
    if (covered != Pc.volume()) return false;
  }
  return true;
}

static sh_status build_links(sh_hierarchy h, int l) {
  // plans between level l-1 (coarse) and l (fine), and the coarse level's covered mask
  Level& F = h->lev[l];
  Level& C = h->lev[l - 1];
  std::vector<InterpSeg> is;
  std::vector<AvgSeg> as;
  std::vector<long long> nc, nc5;
  if (!build_a2(F, C, stencil_depth(h->p), interp_reach(h->p), is, nc) || !build_a5(F, C, as, nc5)) {
    F.stale = true;
    F.a2.release();
    F.a5.release();
    return fail(SH_ENEST, "level " + std::to_string(l) + " is not nested in level " + std::to_string(l - 1));
  }
  HIPCHK(F.a2.upload(is, nc));
  HIPCHK(F.a5.upload(as, nc5));
  F.stale = false;
  HIPCHK(hipMemsetAsync(C.covered(), 0, (size_t)C.g.nvalid, h->st));
  sh_launch_mark_covered(F.a5.segs.p, F.a5.blocks.p, F.a5.nblocks(), C.dbox.p, C.covered(), h->st);
  LAUNCHCHK();
  return SH_OK;
}

// ---------------------------------------------------------------------------------
// Level step pieces
// ---------------------------------------------------------------------------------
// Same-level ghost copy of `role`: one layer, or (deep = true) the whole ghost depth.
// The deep copy carries all four components: the fused step computes its early stages
// on the ghost ring, where it needs Pi as well as psi.
// ncomp 0: the components the stencils read (psi, and Pi under dissipation).
// Debug mode: before a fill that sets every ghost cell of buffer `role` (a stage input
// between stages; U_n at a step's end), NaN into the shell for the components the fill
// carries, so that a ghost a stencil reads but no fill writes shows up as NaN in valid
// cells.
static void poison_before_fill(sh_hierarchy h, int l, int role, int ncomp) {
  if (!(h->debug & 1)) return;
  Level& L = h->lev[l];
  int nz = 0;
  for (const BoxDev& b : L.hbox) nz = std::max(nz, b.nz);
  sh_launch_poison_ghosts(h->p.prec, L.dbox.p, (int)L.hbox.size(), nz + 2 * L.g.ng, L.g.ng, role, ncomp, h->st);
}

static sh_status same_level_fill(sh_hierarchy h, int l, int role, int ncomp = 0, bool deep = true) {
  Level& L = h->lev[l];
  h->rec(2, l, role, 0);
  const bool use_deep = deep && L.a1d.nblocks();
  const SegPlan<CopySeg, SH_WAVE>& pl = use_deep ? L.a1d : L.a1;
  if (ncomp == 0) ncomp = fill_comps(h->p);
  if (use_deep) ncomp = 4;
  hipEvent_t ev = h->prof_begin();
  sh_launch_ghost_copy(h->p.prec, pl.segs.p, pl.blocks.p, pl.nblocks(), L.dbox.p, role, ncomp, h->st);
  h->prof_end(ev, 4);
  LAUNCHCHK();
  return SH_OK;
}

static sh_status coarse_fine_fill(sh_hierarchy h, int l, int role, int anum) {
  if (l == 0) return SH_OK;
  Level& L = h->lev[l];
  h->rec(3, l, role, anum);
  hipEvent_t ev = h->prof_begin();
  sh_launch_ghost_interp(h->p.prec, interp_of(h->p), L.a2.segs.p, L.a2.blocks.p, L.a2.nblocks(), L.dbox.p, h->lev[l - 1].dbox.p, role,
                         anum, fill_comps(h->p), h->st);
  h->prof_end(ev, 5);
  LAUNCHCHK();
  return SH_OK;
}

// Ghost fill of a stage input (one layer suffices: only the state U_n is read deeper).
static sh_status fill(sh_hierarchy h, int l, int role, int anum) {
  poison_before_fill(h, l, role, (role == ROLE_UN && h->lev[l].a1d.nblocks()) ? 4 : fill_comps(h->p));
  sh_status s = same_level_fill(h, l, role, fill_comps(h->p), role == ROLE_UN);
  if (s != SH_OK) return s;
  return coarse_fine_fill(h, l, role, anum);
}

static void stage(sh_hierarchy h, Level& L, int s) {
  const int prec = h->p.prec;
  const bool nt = h->tune.nt != 0;
  const int order = lap_order_of(h->p), ko = ko_of(h->p);
  if (L.stiles_b.n)
    sh_launch_stage(prec, s, h->tune.kind, nt, order, ko, L.stiles_b.p, (int)L.stiles_b.n, L.dbox.p, h->st);
  if (L.stiles_w.n) sh_launch_stage(prec, s, 0, nt, order, ko, L.stiles_w.p, (int)L.stiles_w.n, L.dbox.p, h->st);
}

static sh_status check_level(sh_hierarchy h, int l) {
  if (!h) return fail(SH_EINVAL, "null handle");
  if (l < 0 || l >= (int)h->lev.size()) return fail(SH_EINVAL, "no such level");
  if (h->lev[l].stale) return fail(SH_ESTATE, "level layout must be set again after its coarse level changed");
  return SH_OK;
}

// Calls that synchronise, allocate, upload tables or read back results cannot be
// recorded into a graph.
static sh_status not_capturing(sh_hierarchy h) {
  if (!h) return fail(SH_EINVAL, "null handle");
  if (h->capturing) return fail(SH_ESTATE, "not allowed while a graph is being captured");
  return SH_OK;
}

struct sh_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t st = nullptr;
  struct Adv {
    sh_hierarchy h;
    int level;
    long long dk;
    long long version;
  };
  std::vector<Adv> adv;  // host step counters a replay advances
};

static void shadow_release(sh_hierarchy h);

// ---------------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------------
extern "C" {

const char* sh_last_error(void) { return g_err.c_str(); }

static sh_status check_params(const sh_params* p) {
  if (!p) return fail(SH_EINVAL, "null params");
  if (p->n0 < 1 || !(p->L > 0) || !(p->cfl > 0) || p->beta_pot < 0 || p->max_level < 0 || p->max_level > 15 ||
      p->blocking_factor < 2 || (p->blocking_factor & 1) || p->max_box < p->blocking_factor || p->n_error_buf < 0 ||
      (p->prec != SH_F64 && p->prec != SH_F32))
    return fail(SH_EINVAL, "invalid parameters");
  if (p->integrator != 0 && p->integrator != 3 && p->integrator != 4 && p->integrator != 10 && p->integrator != 21 &&
      p->integrator != 22)
    return fail(SH_EINVAL, "integrator must be 0 or 4 (RK4), 3 or 10 (SSPRK3), 21 (RKN4) or 22 (RKN5)");
  if ((p->integrator == 21 || p->integrator == 22) && (p->alpha_fric != 0.0 || p->ko_order != 0))
    return fail(SH_EINVAL, "RKN4 and RKN5 integrate the friction-free EOM only (alpha_fric = 0, no dissipation)");
  if (p->integrator == 22 && p->max_level != 0)
    return fail(SH_EINVAL, "RKN5 runs on single periodic levels only (max_level = 0)");
  if (p->lap_order < 0 || p->lap_order > 3) return fail(SH_EINVAL, "lap_order must be 0..3");
  if (p->interp != 0 && p->interp != 1 && p->interp != 4) return fail(SH_EINVAL, "interp must be 0, 1 or 4");
  if ((p->ko_order != 0 && p->ko_order != 2 && p->ko_order != 3) || !(p->ko_eps >= 0) || p->ko_eps == HUGE_VAL)
    return fail(SH_EINVAL, "ko_order must be 0, 2 or 3 and ko_eps finite and >= 0");
  if ((long long)p->n0 << p->max_level > 32767) return fail(SH_EINVAL, "finest level too large");
  if (p->tee_fields != 0 && p->tee_fields != 1) return fail(SH_EINVAL, "tee_fields must be 0 or 1");
  return SH_OK;
}

size_t sh_arena_bytes(const sh_params* p, int32_t lev, int32_t nboxes, const int32_t* boxes) {
  if (check_params(p) != SH_OK || lev < 0 || lev > p->max_level) return 0;
  std::vector<IBox> b;
  if (parse_boxes(*p, lev, nboxes, boxes, b) != SH_OK) return 0;
  LayoutGeom g;
  make_geom(p->prec, lev == 0 ? SH_NG0 : refined_ng(*p), b, g, needs_acc(*p), tee_comps(*p));
  return g.total;
}

// ---------------------------------------------------------------------------------
// Staging of the compacted tag list for callers that cannot allocate (see
// sh_tag_cells_noalloc): a fixed device array instead of a buffer grown with hipMalloc.
// Each device holds its own copy until the process ends; host code must use the
// address hipGetSymbolAddress returns for the current device, never the array's name.
// ---------------------------------------------------------------------------------
#define SH_NOALLOC_TAG_CAP (1 << 20)  // tagged cells: 12 MiB of int32 (x, y, z) triplets
static __device__ __align__(256) int32_t scratch[3 * SH_NOALLOC_TAG_CAP];
#define SH_MAX_DEVICES 64
static int32_t* g_scratch_dev[SH_MAX_DEVICES];
static std::mutex g_scratch_mu;

// Device address of `scratch` on device `dev`, looked up once per device with that
// device current (at hierarchy creation).
static sh_status scratch_setup(int dev) {
  if (dev < 0 || dev >= SH_MAX_DEVICES) return fail(SH_EDEVICE, "device index beyond the supported range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return SH_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(SH_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_dev[dev] = (int32_t*)ptr;
  return SH_OK;
}

sh_status sh_hierarchy_create(const sh_params* p, void* hip_stream, sh_hierarchy* out) {
  if (!out) return fail(SH_EINVAL, "null output");
  *out = nullptr;
  sh_status s = check_params(p);
  if (s != SH_OK) return s;
  int ndev = 0;
  const hipError_t de = hipGetDeviceCount(&ndev);
  if (de != hipSuccess || ndev < 1)
    return fail(SH_EDEVICE, std::string("no HIP device (hipGetDeviceCount: ") + hipGetErrorString(de) + ")");
  sh_hierarchy h = new (std::nothrow) sh_hierarchy_s;
  if (!h) return fail(SH_ENOMEM, "host allocation failed");
  h->p = *p;
  h->tune = default_tuning(*p);
  tuning_from_env(h->tune);
  h->st = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->dev) != hipSuccess || scratch_setup(h->dev) != SH_OK) {
    delete h;
    return fail(SH_EDEVICE, "device set-up failed: " + g_err);
  }
  if (hipMalloc((void**)&h->d_ls, (SH_SHADOW_LS + 1) * sizeof(LevelScal)) != hipSuccess ||
      hipMalloc((void**)&h->d_dbg, 16 * sizeof(double)) != hipSuccess) {
    if (h->d_ls) (void)hipFree(h->d_ls);
    delete h;
    return fail(SH_EDEVICE, "device allocation of level scalars failed");
  }
  *out = h;
  return SH_OK;
}

sh_status sh_hierarchy_destroy(sh_hierarchy h) {
  if (!h) return SH_OK;
  if (h->capturing) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(h->st, &g);
    if (g) (void)hipGraphDestroy(g);
  }
  (void)hipStreamSynchronize(h->st);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  shadow_release(h);
  for (Level& L : h->lev) L.release();
  if (h->d_ls) (void)hipFree(h->d_ls);
  if (h->d_dbg) (void)hipFree(h->d_dbg);
  if (h->d_oct) (void)hipFree(h->d_oct);
  if (h->stage.buf) (void)hipHostFree(h->stage.buf);
  delete h;
  return SH_OK;
}

// Scope of one layout change: uploads go through the hierarchy's staging buffer; at the
// end (every return path) the stream is synchronised if anything was queued, and the
// buffer grows to what the change asked for, for the next one.  A hierarchy whose layout
// is set once (an ensemble job) never allocates it.
struct StageScope {
  sh_hierarchy h;
  explicit StageScope(sh_hierarchy h_) : h(h_) {
    h->stage.st = h->st;
    h->stage.used = 0;
    h->stage.want = 0;
    h->stage.queued = false;
    g_stage = &h->stage;
  }
  ~StageScope() {
    g_stage = nullptr;
    UploadStage& sg = h->stage;
    if (sg.queued) (void)hipStreamSynchronize(h->st);
    sg.queued = false;
    sg.used = 0;
    if (sg.want > sg.cap && h->layout_version >= 2) {
      if (sg.buf) (void)hipHostFree(sg.buf);
      sg.buf = nullptr;
      sg.cap = 0;
      const size_t cap = std::max(sg.want + sg.want / 2, (size_t)(1 << 20));
      if (hipHostMalloc((void**)&sg.buf, cap, hipHostMallocDefault) == hipSuccess) sg.cap = cap;
      else sg.buf = nullptr;
    }
  }
};

int32_t sh_num_levels(sh_hierarchy h) { return h ? (int32_t)h->lev.size() : 0; }

static sh_status set_box_tables(sh_hierarchy h, LevelScal* ls, Level& L) {
  L.hbox.clear();
  std::vector<long long> xv{0}, xg{0}, ro{0};
  long long moff = 0;
  for (size_t i = 0; i < L.boxes.size(); ++i) {
    const IBox& b = L.boxes[i];
    BoxDev d;
    for (int s = 0; s < 3; ++s) d.slot[s] = L.base + L.g.off_slot[s] + (size_t)L.g.box_off[i] * L.g.esize;
    d.acc = needs_acc(h->p) ? (double*)(L.base + L.g.off_acc) + L.g.box_off[i] : nullptr;
    d.ls = ls;
    d.cs = L.g.cs[i];
    d.nx = b.size(0);
    d.ny = b.size(1);
    d.nz = b.size(2);
    d.px = L.g.px[i];
    d.py = d.ny + 2 * L.g.ng;
    for (int k = 0; k < 3; ++k) d.lo[k] = b.lo[k];
    if (moff > 0x7fffffffLL) return fail(SH_EINVAL, "level too large for 32-bit mask offsets");
    d.mask_off = (int)moff;
    d.ng = L.g.ng;
    d.xoff = L.g.xoff;
    moff += (long long)d.nx * d.ny * d.nz;
    L.hbox.push_back(d);
    xv.push_back(xv.back() + 4LL * d.nx * d.ny * d.nz);
    xg.push_back(xg.back() + 4LL * (d.nx + 2) * (d.ny + 2) * (d.nz + 2));
    ro.push_back(ro.back() + 4LL * d.nx * d.ny * d.nz);
  }
  ro.pop_back();
  HIPCHK(L.dbox.upload(L.hbox));
  HIPCHK(L.tiles.upload(L.g.tiles));
  {
    std::vector<Tile> wt, bt, ft;
    make_stage_tiles(L.boxes, h->tune, L.g.nvalid, wt, bt);
    HIPCHK(L.stiles_w.upload(wt));
    HIPCHK(L.stiles_b.upload(bt));
    if (fusable(h->p)) make_fused_tiles(L.boxes, h->tune, L.g.ng, ft);
    HIPCHK(L.ftiles.upload(ft));
  }
  HIPCHK(L.xoff_valid.upload(xv));
  HIPCHK(L.xoff_ghost.upload(xg));
  HIPCHK(L.rhs_off.upload(ro));
  return SH_OK;
}

sh_status sh_set_level_layout(sh_hierarchy h, int32_t l, int32_t nboxes, const int32_t* boxes, void* arena,
                              size_t arena_bytes) {
  if (!h) return fail(SH_EINVAL, "null handle");
  if (h->capturing) return not_capturing(h);
  StageScope staged(h);
  h->layout_version += 1;
  const sh_params& p = h->p;
  if (l < 0 || l > p.max_level || l > (int)h->lev.size()) return fail(SH_EINVAL, "bad level");
  if (nboxes == 0) {
    if (l == 0) return fail(SH_EINVAL, "level 0 needs boxes");
    HIPCHK(hipStreamSynchronize(h->st));
    for (size_t i = l; i < h->lev.size(); ++i) h->lev[i].release();
    h->lev.resize(l);
    if (l >= 1) HIPCHK(hipMemsetAsync(h->lev[l - 1].covered(), 0, (size_t)h->lev[l - 1].g.nvalid, h->st));
    return SH_OK;
  }
  if (l > 0 && h->lev[l - 1].stale) return fail(SH_ESTATE, "coarse level layout is stale");
  Level N;
  N.M = p.n0 << l;
  N.dx = level_dx(p, l);
  N.dt = p.cfl * N.dx;
  sh_status s = parse_boxes(p, l, nboxes, boxes, N.boxes);
  if (s != SH_OK) return s;
  if (l == 0) {
    long long v = 0;
    for (auto& b : N.boxes) v += b.volume();
    if (v != (long long)N.M * N.M * N.M) return fail(SH_EINVAL, "level 0 boxes must cover the domain");
  }
  make_geom(p.prec, l == 0 ? SH_NG0 : refined_ng(p), N.boxes, N.g, needs_acc(p), tee_comps(p));
  if (!arena || arena_bytes < N.g.total) return fail(SH_ENOMEM, "arena smaller than sh_arena_bytes");
  N.base = (char*)round_up((long long)(uintptr_t)arena, 256);
  N.bins.build(N.boxes, N.M);
  const bool existing = l < (int)h->lev.size();
  N.k = existing ? h->lev[l].k : (l == 0 ? 0 : 2 * h->lev[l - 1].k);

  s = set_box_tables(h, h->d_ls + l, N);
  if (s != SH_OK) { N.release(); return s; }
  {
    std::vector<CopySeg> cs;
    std::vector<long long> nc;
    // stage inputs: a shell as deep as the stencil; the state after a step: the whole
    // shell (level 0's is deeper, for the fused step)
    const int r = stencil_depth(h->p);
    build_a1(N, r, cs, nc);
    hipError_t e = N.a1.upload(cs, nc);
    if (e == hipSuccess && N.g.ng > r) {
      build_a1(N, N.g.ng, cs, nc);
      e = N.a1d.upload(cs, nc);
    }
    if (e != hipSuccess) { N.release(); return fail(SH_EDEVICE, "table upload failed"); }
  }
  // nesting and interpolation plans against the coarse level
  SegPlan<InterpSeg> fresh;  // valid cells to interpolate from the coarse level
  if (l > 0) {
    const Level& C = h->lev[l - 1];
    std::vector<InterpSeg> is;
    std::vector<long long> nc;
    std::vector<IBox> rem_all;
    for (int d = 0; d < (int)N.boxes.size(); ++d) {
      std::vector<IBox> rem{N.boxes[d]};
      if (existing) {
        const Level& O = h->lev[l];
        O.bins.query(N.boxes[d], [&](int o) {
          std::vector<IBox> nxt;
          for (const IBox& r : rem) subtract(r, O.boxes[o], nxt);
          rem.swap(nxt);
        });
      }
      for (const IBox& R : rem)
        if (!interp_segs(N, C, d, R, interp_reach(p), is, nc)) {
          N.release();
          return fail(SH_ENEST, "level " + std::to_string(l) + " not nested in level " + std::to_string(l - 1));
        }
    }
    if (fresh.upload(is, nc) != hipSuccess) { N.release(); return fail(SH_EDEVICE, "table upload failed"); }
  }
  // copy plan from the old layout
  SegPlan<CopySeg> keep;
  if (existing) {
    const Level& O = h->lev[l];
    std::vector<CopySeg> cs;
    std::vector<long long> nc;
    for (int d = 0; d < (int)N.boxes.size(); ++d)
      O.bins.query(N.boxes[d], [&](int o) {
        const IBox R = isect(N.boxes[d], O.boxes[o]);
        if (R.empty()) return;
        CopySeg c;
        c.dbox = d;
        c.sbox = o;
        for (int k = 0; k < 3; ++k) {
          c.dlo[k] = R.lo[k] - N.boxes[d].lo[k];
          c.slo[k] = R.lo[k] - O.boxes[o].lo[k];
          c.n[k] = R.size(k);
        }
        c.pad = 0;
        cs.push_back(c);
        nc.push_back(R.volume());
      });
    if (keep.upload(cs, nc) != hipSuccess) { N.release(); fresh.release(); return fail(SH_EDEVICE, "table upload failed"); }
  }
  // level scalars (k unchanged for an existing level; a new level starts at its parent's time)
  if (!existing) h->lev.push_back(Level());
  Level old = h->lev[l];
  h->lev[l] = N;
  s = upload_ls(h, l);
  if (s != SH_OK) return s;
  // truncation error estimates: 0 for new cells, kept cells keep theirs
  HIPCHK(hipMemsetAsync(N.tee(), 0, (size_t)N.g.nvalid * 8 * N.g.tee_nc, h->st));
  if (existing) {
    sh_launch_regrid_copy(p.prec, keep.segs.p, keep.blocks.p, keep.nblocks(), N.dbox.p, old.dbox.p, old.tee(),
                          N.tee(), N.g.tee_nc, old.g.nvalid, N.g.nvalid, h->st);
    LAUNCHCHK();
  }
  if (l > 0) {
    // the slopes of the interpolation read the coarse level's same-level ghosts of all
    // four components (the stepping path keeps only the psi pair there)
    s = same_level_fill(h, l - 1, ROLE_UN, 4);
    if (s != SH_OK) return s;
    sh_launch_ghost_interp(p.prec, interp_of(p), fresh.segs.p, fresh.blocks.p, fresh.nblocks(), N.dbox.p, h->lev[l - 1].dbox.p,
                           ROLE_UN, 4, 4, h->st);
    LAUNCHCHK();
  }
  HIPCHK(hipMemsetAsync(N.covered(), 0, (size_t)N.g.nvalid, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  keep.release();
  fresh.release();
  if (existing) old.release();
  if (l > 0) {
    s = build_links(h, l);
    if (s != SH_OK) return s;
  }
  if (l + 1 < (int)h->lev.size()) {
    s = build_links(h, l + 1);
    if (s != SH_OK && s != SH_ENEST) return s;
  }
  // ghosts of the new state (level 0: only meaningful once state is written)
  s = fill(h, l, ROLE_UN, 4);
  if (s != SH_OK) return s;
  HIPCHK(hipStreamSynchronize(h->st));
  g_err.clear();
  return SH_OK;
}

static sh_status xfer(sh_hierarchy h, int l, int role, double* buf, int is_device, int g, bool to_box) {
  sh_status s = check_level(h, l);
  if (s != SH_OK || (s = not_capturing(h)) != SH_OK) return s;
  if (!buf) return fail(SH_EINVAL, "null buffer");
  if (role < 0 || role > 3) return fail(SH_EINVAL, "bad role");
  Level& L = h->lev[l];
  const DevArr<long long>& off = g ? L.xoff_ghost : L.xoff_valid;
  long long total = 0;
  for (const BoxDev& b : L.hbox)
    total += 4LL * (b.nx + 2 * g) * (b.ny + 2 * g) * (b.nz + 2 * g);
  double* dev = buf;
  if (!is_device) {
    HIPCHK(hipMalloc((void**)&dev, (size_t)total * 8));
    if (to_box) {
      hipError_t e = hipMemcpyAsync(dev, buf, (size_t)total * 8, hipMemcpyHostToDevice, h->st);
      if (e != hipSuccess) { (void)hipFree(dev); return fail(SH_EDEVICE, hipGetErrorString(e)); }
    }
  }
  sh_launch_xfer(h->p.prec, to_box, L.dbox.p, off.p, (int)L.hbox.size(), dev, role, g, total, h->st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !is_device) {
    if (!to_box) e = hipMemcpyAsync(buf, dev, (size_t)total * 8, hipMemcpyDeviceToHost, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    (void)hipFree(dev);
  }
  if (e != hipSuccess) return fail(SH_EDEVICE, hipGetErrorString(e));
  return SH_OK;
}

sh_status sh_write_state(sh_hierarchy h, int32_t l, int32_t role, const double* src, int32_t src_is_device,
                         int32_t with_ghosts) {
  return xfer(h, l, role, (double*)src, src_is_device, with_ghosts ? 1 : 0, true);
}

sh_status sh_read_state(sh_hierarchy h, int32_t l, int32_t role, double* dst, int32_t dst_is_device,
                        int32_t with_ghosts) {
  return xfer(h, l, role, dst, dst_is_device, with_ghosts ? 1 : 0, false);
}

sh_status sh_fill_ghosts(sh_hierarchy h, int32_t l, int32_t role, int32_t anum) {
  sh_status s = check_level(h, l);
  if (s != SH_OK) return s;
  if (role < 0 || role > 2 || anum < 0 || anum > 4) return fail(SH_EINVAL, "bad role or alpha");
  return fill(h, l, role, anum);
}

sh_status sh_advance_level(sh_hierarchy h, int32_t l, int32_t sub) {
  sh_status s = check_level(h, l);
  if (s != SH_OK) return s;
  if (l > 0 && sub != 0 && sub != 1) return fail(SH_EINVAL, "substep must be 0 or 1");
  if (l == 0) sub = 0;
  Level& L = h->lev[l];
  hipEvent_t ev;
  if (L.ftiles.n) {
    // all stages in one kernel: no ghost fill between stages is needed because the
    // kernel computes the early stages on the ghost-deep ring itself
    const int nst = stages_of(h->p);
    for (int st = 0; st < nst; ++st) h->rec(1, l, st, sub);
    ev = h->prof_begin();
    sh_launch_fused(h->p.prec, h->tune.nt != 0, h->tune.fshape, h->tune.fvar, nst, L.ftiles.p, (int)L.ftiles.n,
                    L.dbox.p, h->st);
    h->prof_end(ev, 7);
    LAUNCHCHK();
    sh_launch_counter_inc(h->d_ls + l, 1, h->st);
    LAUNCHCHK();
    L.k += 1;
    poison_before_fill(h, l, ROLE_UN, L.a1d.nblocks() ? 4 : fill_comps(h->p));
    return same_level_fill(h, l, ROLE_UN);
  }
  if (rkn5_of(h->p)) {
    // RKN5 (level 0 only): stage inputs U_n, A, B, A; their same-level ghosts are filled
    // before stages 2-4 (no coarse level to interpolate from)
    const int in_role[4] = {ROLE_UN, ROLE_A, ROLE_B, ROLE_A};
    for (int j = 0; j < 4; ++j) {
      if (j > 0 && (s = fill(h, l, in_role[j], 0)) != SH_OK) return s;
      h->rec(1, l, j, sub);
      ev = h->prof_begin();
      stage(h, L, stage_id(h->p, j));
      h->prof_end(ev, j);
      LAUNCHCHK();
    }
  } else if (stages_of(h->p) == 3) {
    // three-stage methods: stage inputs A and B at c = 1 and 1/2 (SSPRK3) or 1/2 and 1
    // (RKN4); alpha in quarters 2 sub + 2 c_s
    for (int j = 0; j < 3; ++j) {
      const int id = stage_id(h->p, j);
      if (j > 0 && (s = fill(h, l, j == 1 ? ROLE_A : ROLE_B, 2 * sub + (int)(2.0 * stage_frac(id)))) != SH_OK)
        return s;
      h->rec(1, l, j, sub);
      ev = h->prof_begin();
      stage(h, L, id);
      h->prof_end(ev, j);
      LAUNCHCHK();
    }
  } else {
    // stage 1 reads U_n (ghosts set by the previous step end or synchronisation)
    h->rec(1, l, 0, sub);
    ev = h->prof_begin();
    stage(h, L, 0);
    h->prof_end(ev, 0);
    LAUNCHCHK();
    // alpha in quarters: (sub + c_s)/2 * 4 = 2 sub + 2 c_s
    if ((s = fill(h, l, ROLE_A, 2 * sub + 1)) != SH_OK) return s;
    h->rec(1, l, 1, sub);
    ev = h->prof_begin();
    stage(h, L, 1);
    h->prof_end(ev, 1);
    LAUNCHCHK();
    if ((s = fill(h, l, ROLE_B, 2 * sub + 1)) != SH_OK) return s;
    h->rec(1, l, 2, sub);
    ev = h->prof_begin();
    stage(h, L, 2);
    h->prof_end(ev, 2);
    LAUNCHCHK();
    if ((s = fill(h, l, ROLE_A, 2 * sub + 2)) != SH_OK) return s;
    h->rec(1, l, 3, sub);
    ev = h->prof_begin();
    stage(h, L, 3);
    h->prof_end(ev, 3);
    LAUNCHCHK();
  }
  sh_launch_counter_inc(h->d_ls + l, 1, h->st);
  LAUNCHCHK();
  L.k += 1;
  poison_before_fill(h, l, ROLE_UN, L.a1d.nblocks() ? 4 : fill_comps(h->p));
  if ((s = same_level_fill(h, l, ROLE_UN)) != SH_OK) return s;
  if (l > 0 && sub == 0) return coarse_fine_fill(h, l, ROLE_UN, 2);
  return SH_OK;
}

sh_status sh_average_down(sh_hierarchy h, int32_t f) {
  sh_status s = check_level(h, f);
  if (s != SH_OK) return s;
  if (f < 1) return fail(SH_EINVAL, "fine level must be >= 1");
  Level& F = h->lev[f];
  Level& C = h->lev[f - 1];
  if (F.k != 2 * C.k) return fail(SH_ESTATE, "levels are not at the same time");
  h->rec(4, f, 0, 0);
  hipEvent_t ev = h->prof_begin();
  sh_launch_avgdown(h->p.prec, F.a5.segs.p, F.a5.blocks.p, F.a5.nblocks(), C.dbox.p, F.dbox.p,
                    h->tee_on ? F.tee() : nullptr, F.g.tee_nc, F.g.nvalid, 1, h->st);
  h->prof_end(ev, 6);
  LAUNCHCHK();
  if ((s = same_level_fill(h, f - 1, ROLE_UN)) != SH_OK) return s;
  return coarse_fine_fill(h, f, ROLE_UN, 4);
}

sh_status sh_set_tee(sh_hierarchy h, int32_t enable, double te_crit, int32_t tag_mode) {
  sh_status s = not_capturing(h);
  if (s != SH_OK) return s;
  if (tag_mode < 1 || tag_mode > 3 || !(te_crit >= 0) || te_crit == HUGE_VAL)
    return fail(SH_EINVAL, "tag_mode must be 1, 2 or 3 and te_crit finite and >= 0");
  h->tee_on = enable != 0;
  for (int c = 0; c < 4; ++c) {
    h->te.crit[c] = te_crit;
    h->te.scale[c] = 1.0;
  }
  h->tag_mode = tag_mode;
  return SH_OK;
}

sh_status sh_set_tee_fields(sh_hierarchy h, int32_t enable, const double* te_crit, const double* scale,
                            int32_t tag_mode) {
  sh_status s = not_capturing(h);
  if (s != SH_OK) return s;
  if (!h->p.tee_fields) return fail(SH_ESTATE, "the hierarchy keeps one estimate per cell (sh_params.tee_fields = 0)");
  if (!te_crit || tag_mode < 1 || tag_mode > 3) return fail(SH_EINVAL, "tag_mode must be 1, 2 or 3 and te_crit given");
  for (int c = 0; c < 4; ++c) {
    const double sc = scale ? scale[c] : 1.0;
    if (!(te_crit[c] >= 0) || te_crit[c] == HUGE_VAL || !(sc >= 0) || sc == HUGE_VAL)
      return fail(SH_EINVAL, "thresholds and scales must be finite and >= 0");
  }
  h->tee_on = enable != 0;
  for (int c = 0; c < 4; ++c) {
    h->te.crit[c] = te_crit[c];
    h->te.scale[c] = scale ? scale[c] : 1.0;
  }
  h->tag_mode = tag_mode;
  return SH_OK;
}

sh_status sh_field_absmax(sh_hierarchy h, double* out_host) {
  if (!h || !out_host) return fail(SH_EINVAL, "null argument");
  if (h->capturing) return not_capturing(h);
  if (h->lev.empty()) return fail(SH_ESTATE, "no levels");
  const int nl = (int)h->lev.size();
  for (int l = 0; l < nl; ++l) {
    Level& L = h->lev[l];
    if (L.stale) return fail(SH_ESTATE, "stale level");
    sh_launch_absmax(h->p.prec, L.tiles.p, L.ntiles(), L.dbox.p, (double*)L.epart(), L.eout(), h->st);
    LAUNCHCHK();
  }
  std::vector<double> all(4 * nl);
  for (int l = 0; l < nl; ++l)
    HIPCHK(hipMemcpyAsync(&all[4 * l], h->lev[l].eout(), 32, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  for (int c = 0; c < 4; ++c) {
    double m = 0.0;
    for (int l = 0; l < nl; ++l) {
      const double v = all[4 * l + c];
      m = (v > m || v != v) ? v : m;
    }
    out_host[c] = m;
  }
  return SH_OK;
}

static void shadow_release(sh_hierarchy h) {
  if (!h->has_shadow) return;
  (void)hipStreamSynchronize(h->st);
  h->shadow.release();
  h->shadow_a5.release();
  if (h->shadow_arena) (void)hipFree(h->shadow_arena);
  h->shadow_arena = nullptr;
  h->shadow = Level();
  h->has_shadow = false;
}

static void shadow_copy(sh_hierarchy h, int role) {
  Level& S = h->shadow;
  sh_launch_ghost_copy(h->p.prec, S.a1.segs.p, S.a1.blocks.p, S.a1.nblocks(), S.dbox.p, role, fill_comps(h->p),
                       h->st);
}

sh_status sh_shadow_begin(sh_hierarchy h) {
  sh_status s = check_level(h, 0);
  if (s != SH_OK || (s = not_capturing(h)) != SH_OK) return s;
  const sh_params& p = h->p;
  Level& L0 = h->lev[0];
  if (rkn5_of(p)) return fail(SH_EINVAL, "no shadow level with RKN5 (single levels only)");
  if (L0.k % 2) return fail(SH_ESTATE, "the shadow starts when level 0 has taken an even number of steps");
  if (p.n0 % 2) return fail(SH_EINVAL, "the shadow level needs an even coarse size");
  for (const IBox& b : L0.boxes)
    for (int d = 0; d < 3; ++d)
      if ((b.lo[d] & 1) || !(b.hi[d] & 1)) return fail(SH_EINVAL, "level-0 boxes must start and end on even cells");
  shadow_release(h);
  Level S;
  S.M = p.n0 / 2;
  S.dx = level_dx(p, 0) * 2.0;
  S.dt = p.cfl * S.dx;
  S.boxes = {IBox{{0, 0, 0}, {S.M - 1, S.M - 1, S.M - 1}}};
  make_geom(p.prec, stencil_depth(p), S.boxes, S.g, needs_acc(p));
  if (hipMalloc((void**)&h->shadow_arena, S.g.total) != hipSuccess) return fail(SH_ENOMEM, "shadow level allocation");
  S.base = (char*)round_up((long long)(uintptr_t)h->shadow_arena, 256);
  S.bins.build(S.boxes, S.M);
  S.k = L0.k / 2;
  h->shadow = S;
  h->has_shadow = true;
  h->shadow_k0 = S.k;
  Level& Sh = h->shadow;
  if ((s = set_box_tables(h, h->d_ls + SH_SHADOW_LS, Sh)) != SH_OK) {
    shadow_release(h);
    return s;
  }
  std::vector<CopySeg> cs;
  std::vector<long long> nc;
  build_a1(Sh, stencil_depth(p), cs, nc);
  std::vector<AvgSeg> as;
  std::vector<long long> nc5;
  if (!build_a5(L0, Sh, as, nc5)) {
    shadow_release(h);
    return fail(SH_EINVAL, "level 0 does not cover the shadow level");
  }
  if (Sh.a1.upload(cs, nc) != hipSuccess || h->shadow_a5.upload(as, nc5) != hipSuccess) {
    shadow_release(h);
    return fail(SH_EDEVICE, "table upload failed");
  }
  LevelScal ls = make_ls(p, 0, Sh.k);
  ls.dx = Sh.dx;
  ls.dt = Sh.dt;
  ls.inv_dx2 = 1.0 / (Sh.dx * Sh.dx);
  ls.ko = ko_coef(p, Sh.dx);
  HIPCHK(hipMemcpyAsync(h->d_ls + SH_SHADOW_LS, &ls, sizeof(ls), hipMemcpyHostToDevice, h->st));
  // the shadow's state: level 0 averaged onto it, then its periodic ghosts
  sh_launch_avgdown(p.prec, h->shadow_a5.segs.p, h->shadow_a5.blocks.p, h->shadow_a5.nblocks(), Sh.dbox.p,
                    L0.dbox.p, nullptr, 1, 0, 1, h->st);
  LAUNCHCHK();
  shadow_copy(h, ROLE_UN);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(h->st));
  return SH_OK;
}

sh_status sh_shadow_advance(sh_hierarchy h) {
  sh_status s = not_capturing(h);
  if (s != SH_OK) return s;
  if (!h->has_shadow) return fail(SH_ESTATE, "no shadow level");
  Level& S = h->shadow;
  if (S.k != h->shadow_k0) return fail(SH_ESTATE, "the shadow takes a single step");
  // one step of twice the level-0 step on the periodic shadow lattice
  if (stages_of(h->p) == 3) {
    stage(h, S, stage_id(h->p, 0));
    shadow_copy(h, ROLE_A);
    stage(h, S, stage_id(h->p, 1));
    shadow_copy(h, ROLE_B);
    stage(h, S, stage_id(h->p, 2));
  } else {
    stage(h, S, 0);
    shadow_copy(h, ROLE_A);
    stage(h, S, 1);
    shadow_copy(h, ROLE_B);
    stage(h, S, 2);
    shadow_copy(h, ROLE_A);
    stage(h, S, 3);
  }
  sh_launch_counter_inc(h->d_ls + SH_SHADOW_LS, 1, h->st);
  S.k += 1;
  shadow_copy(h, ROLE_UN);
  LAUNCHCHK();
  return SH_OK;
}

sh_status sh_shadow_end(sh_hierarchy h) {
  sh_status s = check_level(h, 0);
  if (s != SH_OK || (s = not_capturing(h)) != SH_OK) return s;
  if (!h->has_shadow) return fail(SH_ESTATE, "no shadow level");
  Level& L0 = h->lev[0];
  Level& S = h->shadow;
  if (S.k != h->shadow_k0 + 1 || L0.k != 2 * S.k) {
    return fail(SH_ESTATE, "level 0 and the shadow are not at the same time after one shadow step");
  }
  // estimate on level 0: shadow against level 0 averaged, the shadow itself unchanged
  sh_launch_avgdown(h->p.prec, h->shadow_a5.segs.p, h->shadow_a5.blocks.p, h->shadow_a5.nblocks(), S.dbox.p,
                    L0.dbox.p, L0.tee(), L0.g.tee_nc, L0.g.nvalid, 0, h->st);
  LAUNCHCHK();
  shadow_release(h);
  return SH_OK;
}

sh_status sh_read_tee(sh_hierarchy h, int32_t l, double* out_dev) {
  sh_status s = check_level(h, l);
  if (s != SH_OK || (s = not_capturing(h)) != SH_OK) return s;
  if (!out_dev) return fail(SH_EINVAL, "null output");
  const Level& L = h->lev[l];
  HIPCHK(hipMemcpyAsync(out_dev, L.tee(), (size_t)L.g.nvalid * 8 * L.g.tee_nc, hipMemcpyDeviceToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return SH_OK;
}

// Tagging of a level; the compacted list is staged in `staging` (device memory with room
// for `cap` cells, checked by the caller) when given, else in the level's own buffer,
// grown with hipMalloc as needed.
static sh_status compact_tags(sh_hierarchy h, int32_t l, const uint8_t* mask, int32_t* idx_host, long long want,
                              int32_t* staging);

static sh_status tag_cells(sh_hierarchy h, int32_t l, uint8_t* mask_dev, int32_t* idx_host, int64_t cap,
                           int64_t* ntag, int32_t* staging) {
  sh_status s = check_level(h, l);
  if (s != SH_OK || (s = not_capturing(h)) != SH_OK) return s;
  if (cap < 0) return fail(SH_EINVAL, "negative capacity");
  Level& L = h->lev[l];
  if ((s = fill(h, l, ROLE_UN, 4)) != SH_OK) return s;
  uint8_t* mask = mask_dev ? mask_dev : L.mask();
  const int nt = L.ntiles();
  TeeSpec te = h->te;
  te.nc = L.g.tee_nc;
  te.cs = L.g.nvalid;
  sh_launch_tag(h->p.prec, L.tiles.p, nt, L.dbox.p, mask, L.tile_count(), L.tee(), te, h->tag_mode, h->st);
  LAUNCHCHK();
  sh_launch_scan(L.tile_count(), L.tile_off(), nt, h->st);
  LAUNCHCHK();
  long long total = 0;
  HIPCHK(hipMemcpyAsync(&total, L.tile_off() + nt, 8, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  if (ntag) *ntag = total;
  return compact_tags(h, l, mask, idx_host, std::min<long long>(total, cap), staging);
}

// The first `want` tagged cells of the mask just computed by tag_cells (its tile offsets
// are current), as (x, y, z) triples into idx_host.
static sh_status compact_tags(sh_hierarchy h, int32_t l, const uint8_t* mask, int32_t* idx_host, long long want,
                              int32_t* staging) {
  Level& L = h->lev[l];
  const int nt = L.ntiles();
  if (idx_host && want > 0) {
    int32_t* idx = staging;
    if (!idx) {
      if (L.d_idx_cap < want) {
        if (L.d_idx) (void)hipFree(L.d_idx);
        L.d_idx = nullptr;
        L.d_idx_cap = 0;
        HIPCHK(hipMalloc((void**)&L.d_idx, (size_t)want * 12));
        L.d_idx_cap = want;
      }
      idx = L.d_idx;
    }
    sh_launch_tag_compact(L.tiles.p, nt, L.dbox.p, mask, L.tile_off(), idx, want, h->st);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(idx_host, idx, (size_t)want * 12, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
  }
  return SH_OK;
}

sh_status sh_tag_cells(sh_hierarchy h, int32_t l, uint8_t* mask_dev, int32_t* idx_host, int64_t cap,
                       int64_t* ntag) {
  return tag_cells(h, l, mask_dev, idx_host, cap, ntag, nullptr);
}

sh_status sh_tag_cells_noalloc(sh_hierarchy h, int32_t l, uint8_t* mask_dev, int32_t* idx_host, int64_t cap,
                               int64_t* ntag) {
  if (!h) return fail(SH_EINVAL, "null handle");
  if (idx_host && cap > SH_NOALLOC_TAG_CAP)
    return fail(SH_EINVAL, "cap " + std::to_string(cap) + " exceeds the allocation-free maximum of " +
                               std::to_string(SH_NOALLOC_TAG_CAP) + " tagged cells");
  if (h->dev < 0 || h->dev >= SH_MAX_DEVICES || !g_scratch_dev[h->dev])
    return fail(SH_ESTATE, "no staging array for the hierarchy's device");
  return tag_cells(h, l, mask_dev, idx_host, cap, ntag, g_scratch_dev[h->dev]);
}

sh_status sh_energy(sh_hierarchy h, double* e_host, int64_t* nonfinite) {
  if (!h || !e_host) return fail(SH_EINVAL, "null argument");
  if (h->capturing) return not_capturing(h);
  if (h->lev.empty()) return fail(SH_ESTATE, "no levels");
  const int nl = (int)h->lev.size();
  for (int l = 0; l < nl; ++l) {
    if (h->lev[l].stale) return fail(SH_ESTATE, "stale level");
    Level& L = h->lev[l];
    const uint8_t* cov = (l + 1 < nl) ? L.covered() : nullptr;
    sh_launch_energy(h->p.prec, L.tiles.p, L.ntiles(), L.dbox.p, cov, L.epart(), h->st);
    LAUNCHCHK();
    sh_launch_energy_final(L.epart(), L.ntiles(), L.dx * L.dx * L.dx, L.eout(), h->st);
    LAUNCHCHK();
  }
  std::vector<double> all(4 * nl);
  for (int l = 0; l < nl; ++l)
    HIPCHK(hipMemcpyAsync(&all[4 * l], h->lev[l].eout(), 32, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  double k = 0, g = 0, pt = 0, bad = 0;
  for (int l = 0; l < nl; ++l) {
    k += all[4 * l];
    g += all[4 * l + 1];
    pt += all[4 * l + 2];
    bad += all[4 * l + 3];
  }
  e_host[0] = k;
  e_host[1] = g;
  e_host[2] = pt;
  e_host[3] = k + g + pt;
  if (nonfinite) *nonfinite = (int64_t)bad;
  return SH_OK;
}

sh_status sh_eval_rhs(sh_hierarchy h, int32_t l, double* out_dev) {
  sh_status s = check_level(h, l);
  if (s != SH_OK || (s = not_capturing(h)) != SH_OK) return s;
  if (!out_dev) return fail(SH_EINVAL, "null output");
  Level& L = h->lev[l];
  sh_launch_rhs(h->p.prec, lap_order_of(h->p), ko_of(h->p), L.tiles.p, L.ntiles(), L.dbox.p, L.rhs_off.p, out_dev, h->st);
  LAUNCHCHK();
  return SH_OK;
}

sh_status sh_level_info(sh_hierarchy h, int32_t l, int64_t* k, double* eta, int32_t* nboxes, int64_t* ncells) {
  if (!h || l < 0 || l >= (int)h->lev.size()) return fail(SH_EINVAL, "no such level");
  const Level& L = h->lev[l];
  if (k) *k = L.k;
  if (eta) *eta = h->p.eta0 + (double)L.k * L.dt;
  if (nboxes) *nboxes = (int32_t)L.boxes.size();
  if (ncells) *ncells = L.g.nvalid;
  return SH_OK;
}

sh_status sh_sync(sh_hierarchy h) {
  if (!h) return fail(SH_EINVAL, "null handle");
  if (h->capturing) return not_capturing(h);
  HIPCHK(hipStreamSynchronize(h->st));
  HIPCHK(hipGetLastError());
  return SH_OK;
}

sh_status sh_set_stream(sh_hierarchy h, void* hip_stream) {
  sh_status s = not_capturing(h);
  if (s != SH_OK) return s;
  h->st = (hipStream_t)hip_stream;
  return SH_OK;
}

sh_status sh_restart(sh_hierarchy h) {
  sh_status s = not_capturing(h);
  if (s != SH_OK) return s;
  if (h->lev.empty()) return fail(SH_ESTATE, "no levels");
  if (h->has_shadow) return fail(SH_ESTATE, "a shadow level is active");
  for (Level& L : h->lev) L.k = 0;
  sh_launch_counter_zero(h->d_ls, (int)h->lev.size(), h->st);
  LAUNCHCHK();
  return SH_OK;
}

sh_status sh_set_debug(sh_hierarchy h, int32_t flags) {
  sh_status s = not_capturing(h);
  if (s != SH_OK) return s;
  if (flags & ~1) return fail(SH_EINVAL, "unknown debug flags");
  h->debug = flags;
  return SH_OK;
}

sh_status sh_stream_probe(int32_t kind, const void* src, void* dst, int64_t bytes, void* hip_stream) {
  if (kind < 0 || kind > 2) return fail(SH_EINVAL, "stream probe kind must be 0 (read), 1 (write) or 2 (copy)");
  if (bytes <= 0 || (bytes & 15)) return fail(SH_EINVAL, "stream probe size must be a positive multiple of 16 bytes");
  if (!dst || (kind != 1 && !src)) return fail(SH_EINVAL, "stream probe needs a destination (and a source to read)");
  if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return fail(SH_EINVAL, "stream probe buffers must be 16-byte aligned");
  const long long nwords = bytes / 16;
  if ((nwords + sh_stream_words_per_block() - 1) / sh_stream_words_per_block() > 0x7fffffffLL)
    return fail(SH_EINVAL, "stream probe size too large for one launch");
  sh_launch_stream(kind, src, dst, nwords, (hipStream_t)hip_stream);
  HIPCHK(hipGetLastError());
  return SH_OK;
}

sh_status sh_debug_stage_scalars(sh_hierarchy h, int32_t l, int32_t s, double* out_host) {
  sh_status st = check_level(h, l);
  if (st != SH_OK || (st = not_capturing(h)) != SH_OK) return st;
  const int nst = stages_of(h->p);
  if (s < 0 || s >= nst || !out_host) return fail(SH_EINVAL, "bad stage");
  sh_launch_debug_scalars(h->d_ls + l, stage_id(h->p, s), h->d_dbg, h->st);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(out_host, h->d_dbg, 7 * 8, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return SH_OK;
}

static sh_status emit_boxes(const std::vector<IBox>& out, int32_t* boxes_out, int32_t cap, int32_t* nboxes) {
  *nboxes = (int32_t)out.size();
  if ((int)out.size() > cap) return fail(SH_ENOMEM, "box capacity too small");
  for (size_t i = 0; i < out.size(); ++i)
    for (int d = 0; d < 3; ++d) {
      boxes_out[6 * i + d] = out[i].lo[d];
      boxes_out[6 * i + 3 + d] = out[i].hi[d];
    }
  return SH_OK;
}

sh_status sh_cluster_boxes(int32_t M, int32_t nlevel_boxes, const int32_t* level_boxes, int32_t bf, int32_t max_box,
                           int32_t n_error_buf, double efficiency, int64_t ntag, const int32_t* tags,
                           int32_t* boxes_out, int32_t cap, int32_t* nboxes) {
  if (M < 1 || nlevel_boxes < 0 || (nlevel_boxes > 0 && !level_boxes) || ntag < 0 || (ntag > 0 && !tags) ||
      !nboxes || cap < 0 || (cap > 0 && !boxes_out) || !(efficiency > 0) || efficiency > 1 || n_error_buf < 0 ||
      max_box < bf)
    return fail(SH_EINVAL, "bad clustering arguments");
  std::vector<IBox> lb;
  for (int i = 0; i < nlevel_boxes; ++i) {
    IBox b;
    for (int d = 0; d < 3; ++d) {
      b.lo[d] = level_boxes[6 * i + d];
      b.hi[d] = level_boxes[6 * i + 3 + d];
    }
    lb.push_back(b);
  }
  std::vector<IBox> out;
  std::string err;
  if (!cluster_level(M, lb, nlevel_boxes == 0, bf, max_box, n_error_buf, efficiency, tags, ntag, out, err))
    return fail(SH_EINVAL, err);
  return emit_boxes(out, boxes_out, cap, nboxes);
}

sh_status sh_cluster_boxes_carried(int32_t M, int32_t nlevel_boxes, const int32_t* level_boxes, int32_t bf,
                                   int32_t max_box, int32_t n_error_buf, double efficiency, int64_t ntag,
                                   const int32_t* tags, int64_t ncarried, const int32_t* carried, int32_t grow,
                                   int32_t* boxes_out, int32_t cap, int32_t* nboxes) {
  if (ncarried < 0 || (ncarried > 0 && !carried) || grow < 0 || grow > M)
    return fail(SH_EINVAL, "bad carried tags");
  if (M < 1 || nlevel_boxes < 0 || (nlevel_boxes > 0 && !level_boxes) || ntag < 0 || (ntag > 0 && !tags) ||
      !nboxes || cap < 0 || (cap > 0 && !boxes_out) || !(efficiency > 0) || efficiency > 1 || n_error_buf < 0 ||
      max_box < bf)
    return fail(SH_EINVAL, "bad clustering arguments");
  std::vector<IBox> lb;
  for (int i = 0; i < nlevel_boxes; ++i) {
    IBox b;
    for (int d = 0; d < 3; ++d) {
      b.lo[d] = level_boxes[6 * i + d];
      b.hi[d] = level_boxes[6 * i + 3 + d];
    }
    lb.push_back(b);
  }
  std::vector<IBox> out;
  std::string err;
  if (!cluster_level(M, lb, nlevel_boxes == 0, bf, max_box, n_error_buf, efficiency, tags, ntag, out, err, carried,
                     ncarried, grow))
    return fail(SH_EINVAL, err);
  return emit_boxes(out, boxes_out, cap, nboxes);
}

static bool read_boxes(int32_t n, const int32_t* in, std::vector<IBox>& out) {
  out.clear();
  if (n < 0 || (n > 0 && !in)) return false;
  for (int i = 0; i < n; ++i) {
    IBox b;
    for (int d = 0; d < 3; ++d) {
      b.lo[d] = in[6 * i + d];
      b.hi[d] = in[6 * i + 3 + d];
    }
    out.push_back(b);
  }
  return true;
}

sh_status sh_local_tag_boxes(int32_t M_fine, int32_t nfine, const int32_t* fine_boxes, int32_t bf, int32_t n_error_buf,
                             int32_t max_box, int64_t ntag, const int32_t* tags, int32_t* boxes_out, int32_t cap,
                             int32_t* nboxes) {
  std::vector<IBox> fb, out;
  if (!read_boxes(nfine, fine_boxes, fb) || ntag < 0 || (ntag > 0 && !tags) || !nboxes || cap < 0 ||
      (cap > 0 && !boxes_out) || n_error_buf < 0 || max_box < bf)
    return fail(SH_EINVAL, "bad local regrid arguments");
  std::string err;
  if (!local_tag_boxes(M_fine, fb, bf, n_error_buf, max_box, tags, ntag, out, err)) return fail(SH_EINVAL, err);
  return emit_boxes(out, boxes_out, cap, nboxes);
}

sh_status sh_local_nest_boxes(int32_t M_level, int32_t nadded, const int32_t* added_fine, int32_t nlevel,
                              const int32_t* level_boxes, int32_t bf, int32_t max_box, int32_t* boxes_out, int32_t cap,
                              int32_t* nboxes) {
  std::vector<IBox> ab, lb, out;
  if (!read_boxes(nadded, added_fine, ab) || !read_boxes(nlevel, level_boxes, lb) || !nboxes || cap < 0 ||
      (cap > 0 && !boxes_out) || max_box < bf)
    return fail(SH_EINVAL, "bad local regrid arguments");
  std::string err;
  if (!local_nest_boxes(M_level, ab, lb, bf, max_box, out, err)) return fail(SH_EINVAL, err);
  return emit_boxes(out, boxes_out, cap, nboxes);
}

sh_status sh_cluster_tags(sh_hierarchy h, int32_t l, int64_t ntag, const int32_t* tags, double efficiency,
                          int32_t* boxes_out, int32_t cap, int32_t* nboxes) {
  sh_status s = check_level(h, l);
  if (s != SH_OK) return s;
  if (ntag < 0 || (ntag > 0 && !tags) || !nboxes || cap < 0 || (cap > 0 && !boxes_out) || !(efficiency > 0) ||
      efficiency > 1)
    return fail(SH_EINVAL, "bad clustering arguments");
  const sh_params& p = h->p;
  const Level& L = h->lev[l];
  std::vector<IBox> out;
  std::string err;
  if (!cluster_level(L.M, L.boxes, l == 0, p.blocking_factor, p.max_box, p.n_error_buf, efficiency, tags, ntag, out,
                     err))
    return fail(SH_EINVAL, err);
  return emit_boxes(out, boxes_out, cap, nboxes);
}

sh_status sh_cluster_tags_carried(sh_hierarchy h, int32_t l, int64_t ntag, const int32_t* tags, int64_t ncarried,
                                  const int32_t* carried, int32_t grow, double efficiency, int32_t* boxes_out,
                                  int32_t cap, int32_t* nboxes) {
  sh_status s = check_level(h, l);
  if (s != SH_OK) return s;
  if (ntag < 0 || (ntag > 0 && !tags) || ncarried < 0 || (ncarried > 0 && !carried) || grow < 0 ||
      grow > h->lev[l].M || !nboxes || cap < 0 || (cap > 0 && !boxes_out) || !(efficiency > 0) || efficiency > 1)
    return fail(SH_EINVAL, "bad clustering arguments");
  const sh_params& p = h->p;
  const Level& L = h->lev[l];
  std::vector<IBox> out;
  std::string err;
  if (!cluster_level(L.M, L.boxes, l == 0, p.blocking_factor, p.max_box, p.n_error_buf, efficiency, tags, ntag, out,
                     err, carried, ncarried, grow))
    return fail(SH_EINVAL, err);
  return emit_boxes(out, boxes_out, cap, nboxes);
}

sh_status sh_tag_blocks(sh_hierarchy h, int32_t l, int32_t halve, int32_t r, uint64_t* bits_host, int64_t nwords,
                        int64_t* ntag) {
  sh_status s = check_level(h, l);
  if (s != SH_OK || (s = not_capturing(h)) != SH_OK) return s;
  if ((halve != 0 && halve != 1) || (halve && l == 0) || r < 0 || !bits_host || nwords < 0)
    return fail(SH_EINVAL, "bad block tagging arguments");
  Level& L = h->lev[l];
  const int bf = h->p.blocking_factor, b = bf / 2;
  const int M = halve ? L.M / 2 : L.M;
  if (nwords != block_words(M, bf)) return fail(SH_EINVAL, "block bitset of the wrong size");
  int bsh = 0;
  while ((1 << bsh) < b) ++bsh;
  int64_t n = 0;
  if ((s = tag_cells(h, l, nullptr, nullptr, 0, &n, nullptr)) != SH_OK) return s;
  if (ntag) *ntag = n;
  if (n == 0) return SH_OK;
  // octant bitsets cost 8 bits per block of the target level to clear, copy and grow, a
  // tag list 12 bytes and a marking step per tag: octants from one tag per 16 blocks on
  const long long nb = M / b;
  const bool octants = (1 << bsh) == b && 2 * r >= b && r < b && n >= nb * nb * nb / 16;
  std::string err;
  if (!octants) {
    std::vector<int32_t> idx((size_t)n * 3);
    if ((s = compact_tags(h, l, L.mask(), idx.data(), n, nullptr)) != SH_OK) return s;
    if (!mark_list_blocks(M, bf, r, halve != 0, idx.data(), n, bits_host, nwords, err)) return fail(SH_EINVAL, err);
    return SH_OK;
  }
  if (h->oct_words < nwords) {
    if (h->d_oct) (void)hipFree(h->d_oct);
    h->d_oct = nullptr;
    h->oct_words = 0;
    HIPCHK(hipMalloc((void**)&h->d_oct, (size_t)8 * nwords * 8));
    h->oct_words = nwords;
  }
  HIPCHK(hipMemsetAsync(h->d_oct, 0, (size_t)8 * nwords * 8, h->st));
  sh_launch_tag_octants(L.tiles.p, L.ntiles(), L.dbox.p, L.mask(), halve, r, bsh, (int)nb, h->d_oct, nwords, h->st);
  LAUNCHCHK();
  h->h_oct.resize((size_t)8 * nwords);
  HIPCHK(hipMemcpyAsync(h->h_oct.data(), h->d_oct, (size_t)8 * nwords * 8, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  if (!dilate_octants(M, bf, h->h_oct.data(), bits_host, nwords, err)) return fail(SH_EINVAL, err);
  return SH_OK;
}

sh_status sh_cluster_blocks(sh_hierarchy h, int32_t l, const uint64_t* bits, int64_t nwords, double efficiency,
                            int32_t* boxes_out, int32_t cap, int32_t* nboxes) {
  sh_status s = check_level(h, l);
  if (s != SH_OK) return s;
  if (!bits || nwords < 0 || !nboxes || cap < 0 || (cap > 0 && !boxes_out) || !(efficiency > 0) || efficiency > 1)
    return fail(SH_EINVAL, "bad clustering arguments");
  const sh_params& p = h->p;
  const Level& L = h->lev[l];
  std::vector<IBox> out;
  std::string err;
  if (!cluster_bits(L.M, L.boxes, l == 0, p.blocking_factor, p.max_box, efficiency, bits, nwords, out, err))
    return fail(SH_EINVAL, err);
  return emit_boxes(out, boxes_out, cap, nboxes);
}

sh_status sh_cluster_boxes_bits(int32_t M, int32_t nlevel_boxes, const int32_t* level_boxes, int32_t bf,
                                int32_t max_box, double efficiency, const uint64_t* bits, int64_t nwords,
                                int32_t* boxes_out, int32_t cap, int32_t* nboxes) {
  std::vector<IBox> lb;
  if (M < 1 || !read_boxes(nlevel_boxes, level_boxes, lb) || !bits || nwords < 0 || !nboxes || cap < 0 ||
      (cap > 0 && !boxes_out) || !(efficiency > 0) || efficiency > 1 || max_box < bf)
    return fail(SH_EINVAL, "bad clustering arguments");
  std::vector<IBox> out;
  std::string err;
  if (!cluster_bits(M, lb, nlevel_boxes == 0, bf, max_box, efficiency, bits, nwords, out, err))
    return fail(SH_EINVAL, err);
  return emit_boxes(out, boxes_out, cap, nboxes);
}

sh_status sh_dilate_octants(int32_t M, int32_t blocking_factor, const uint64_t* octants, uint64_t* bits,
                            int64_t nwords) {
  if (M < 1 || !octants || !bits || nwords < 0) return fail(SH_EINVAL, "bad octant arguments");
  std::string err;
  if (!dilate_octants(M, blocking_factor, octants, bits, nwords, err)) return fail(SH_EINVAL, err);
  return SH_OK;
}

sh_status sh_set_tuning(sh_hierarchy h, int32_t kind, int32_t nontemporal, int32_t tile_z, int32_t fuse,
                        int32_t fused_shape, int32_t fused_tile_z, int32_t fused_variant) {
  if (!h) return fail(SH_EINVAL, "null handle");
  if (h->capturing) return not_capturing(h);
  if ((kind != 0 && kind != 4 && kind != 8) || (nontemporal != 0 && nontemporal != 1) || tile_z < 0 ||
      tile_z > 1024 || (fuse != 0 && fuse != 4) || (fused_shape < 0 || fused_shape > 3) || fused_tile_z < 0 ||
      fused_tile_z > 1024 || fused_variant < 0 || fused_variant > 8)
    return fail(SH_EINVAL, "bad tuning");
  HIPCHK(hipStreamSynchronize(h->st));
  h->tune.kind = kind;
  h->tune.nt = nontemporal;
  h->tune.zc = tile_z;
  h->tune.fuse = fuse;
  h->tune.fshape = fused_shape;
  h->tune.fzc = fused_tile_z;
  h->tune.fvar = fused_variant;
  for (Level& L : h->lev) {
    std::vector<Tile> wt, bt, ft;
    make_stage_tiles(L.boxes, h->tune, L.g.nvalid, wt, bt);
    HIPCHK(L.stiles_w.upload(wt));
    HIPCHK(L.stiles_b.upload(bt));
    if (fusable(h->p)) make_fused_tiles(L.boxes, h->tune, L.g.ng, ft);
    HIPCHK(L.ftiles.upload(ft));
  }
  return SH_OK;
}

sh_status sh_profile(sh_hierarchy h, int32_t enable) {
  if (!h) return fail(SH_EINVAL, "null handle");
  if (h->capturing) return not_capturing(h);
  h->prof_collect();
  h->profiling = enable != 0;
  for (int i = 0; i < 8; ++i) {
    h->prof_ms[i] = 0;
    h->prof_n[i] = 0;
  }
  return SH_OK;
}

sh_status sh_profile_read(sh_hierarchy h, double* ms, int64_t* counts) {
  if (!h || !ms || !counts) return fail(SH_EINVAL, "null argument");
  if (h->capturing) return not_capturing(h);
  h->prof_collect();
  for (int i = 0; i < 8; ++i) {
    ms[i] = h->prof_ms[i];
    counts[i] = h->prof_n[i];
  }
  return SH_OK;
}

sh_status sh_trace(sh_hierarchy h, int32_t enable) {
  if (!h) return fail(SH_EINVAL, "null handle");
  if (h->capturing) return not_capturing(h);
  h->tracing = enable != 0;
  h->trace.clear();
  return SH_OK;
}

int64_t sh_trace_read(sh_hierarchy h, int32_t* out, int64_t cap) {
  if (!h) return -1;
  const int64_t n = (int64_t)h->trace.size() / 4;
  if (out) std::memcpy(out, h->trace.data(), (size_t)std::min(n, cap) * 16);
  return n;
}

sh_status sh_capture_begin(sh_hierarchy h) {
  sh_status s = not_capturing(h);
  if (s != SH_OK) return s;
  if (h->profiling || h->tracing) return fail(SH_ESTATE, "switch profiling and tracing off before capturing");
  if (!h->st) return fail(SH_EINVAL, "the legacy default stream cannot be captured: create the hierarchy on a stream");
  if (h->lev.empty()) return fail(SH_ESTATE, "no levels");
  for (const Level& L : h->lev)
    if (L.stale) return fail(SH_ESTATE, "a level layout is stale");
  HIPCHK(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
  h->k_at_capture.clear();
  for (const Level& L : h->lev) h->k_at_capture.push_back(L.k);
  h->capturing = true;
  return SH_OK;
}

sh_status sh_capture_end(sh_hierarchy h, sh_graph* out) {
  if (!h || !out) return fail(SH_EINVAL, "null argument");
  *out = nullptr;
  if (!h->capturing) return fail(SH_ESTATE, "no capture in progress");
  h->capturing = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->st, &g);
  sh_graph G = new (std::nothrow) sh_graph_s;
  // the captured steps have not run: put the host counters back
  for (size_t l = 0; l < h->lev.size() && l < h->k_at_capture.size(); ++l) {
    const long long dk = h->lev[l].k - h->k_at_capture[l];
    h->lev[l].k = h->k_at_capture[l];
    if (G && dk) G->adv.push_back({h, (int)l, dk, h->layout_version});
  }
  if (e != hipSuccess || !g || !G) {
    if (g) (void)hipGraphDestroy(g);
    delete G;
    return fail(e != hipSuccess ? SH_EDEVICE : SH_ENOMEM, e != hipSuccess ? hipGetErrorString(e) : "capture failed");
  }
  G->graph = g;
  G->st = h->st;
  e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    delete G;
    return fail(SH_EDEVICE, hipGetErrorString(e));
  }
  *out = G;
  return SH_OK;
}

sh_status sh_graph_launch(sh_graph g) {
  if (!g || !g->exec) return fail(SH_EINVAL, "null graph");
  for (const auto& a : g->adv) {
    if (a.h->capturing) return fail(SH_ESTATE, "not allowed while a graph is being captured");
    if (a.h->layout_version != a.version || a.level >= (int)a.h->lev.size())
      return fail(SH_ESTATE, "the layout changed since the graph was captured");
  }
  HIPCHK(hipGraphLaunch(g->exec, g->st));
  for (const auto& a : g->adv) a.h->lev[a.level].k += a.dk;
  return SH_OK;
}

sh_status sh_graph_destroy(sh_graph g) {
  if (!g) return SH_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return SH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Batches: one RK4 step of level 0 of many single-level hierarchies per launch
// ---------------------------------------------------------------------------------
// Batch tables stay allocated while the batch lives: a new member list is planned on the
// host and its tables are copied into the same device buffers in stream order (a launch
// queued before the change still reads the old contents), staged through pinned host
// buffers that rotate so the host waits for none of them in the common case.  Only a
// table that outgrows its buffer makes the change wait for the stream.
template <typename T>
struct DevVec {
  T* p = nullptr;
  size_t n = 0, cap = 0;
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = cap = 0;
  }
};

#define SH_BATCH_STAGES 4
struct BatchStage {
  char* buf = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;  // recorded after the copies out of buf
  bool used = false;
};

struct sh_batch_s {
  std::vector<sh_hierarchy> jobs;
  hipStream_t st = nullptr;
  int prec = 0;
  Tuning tune;
  DevVec<BoxDev> boxes;                // every job's level-0 boxes, job after job
  DevVec<Tile> ftiles;                 // fused-step tiles of the jobs that take the fused path
  DevVec<Tile> wtiles, btiles;         // per-stage tiles of the other jobs
  DevVec<CopySeg> a1s_segs, a1d_segs;  // one-layer ghost copy of the per-stage jobs; full-depth
  DevVec<SegBlock> a1s_blocks, a1d_blocks;  // ghost copy of every job (after the step)
  DevVec<LevelScal*> counters;
  std::vector<long long> versions;  // each job's layout version when the batch was built
  BatchStage stage[SH_BATCH_STAGES];
  int next_stage = 0;
  void release() {
    boxes.release();
    ftiles.release();
    wtiles.release();
    btiles.release();
    a1s_segs.release();
    a1d_segs.release();
    a1s_blocks.release();
    a1d_blocks.release();
    counters.release();
    for (BatchStage& g : stage) {
      if (g.buf) (void)hipHostFree(g.buf);
      if (g.done) (void)hipEventDestroy(g.done);
      g = BatchStage();
    }
  }
};

static std::vector<SegBlock> wave_blocks(const std::vector<long long>& ncell_per_seg) {
  std::vector<SegBlock> b;
  for (size_t i = 0; i < ncell_per_seg.size(); ++i)
    for (long long s = 0; s < ncell_per_seg[i]; s += SH_WAVE) b.push_back(SegBlock{(int)i, (int)s});
  return b;
}

// Plan the tables of a member list and copy them into the batch's buffers.
static sh_status batch_set_jobs(sh_batch b, int njobs, const sh_hierarchy* jobs) {
  std::vector<BoxDev> boxes;
  std::vector<Tile> ft, wt, bt;
  std::vector<CopySeg> s1, sd;
  std::vector<long long> n1, nd, versions;
  std::vector<LevelScal*> ctr;
  // one fused tile depth for the whole batch, from all members' columns together
  long long columns = 0;
  int nz_max = 1;
  for (int j = 0; j < njobs; ++j)
    if (jobs[j] && jobs[j]->lev.size() == 1) {
      const Level& L = jobs[j]->lev[0];
      columns += fused_columns(L.boxes, b->tune, L.g.ng);
      for (const IBox& x : L.boxes) nz_max = std::max(nz_max, x.size(2));
    }
  const int batch_zc = fused_zc(b->tune, columns, nz_max);
  for (int j = 0; j < njobs; ++j) {
    sh_hierarchy h = jobs[j];
    if (!h || h->lev.size() != 1 || h->st != b->st || h->p.prec != b->prec)
      return fail(SH_EINVAL, "batched jobs must be single-level hierarchies of one precision on one stream");
    if (stages_of(h->p) != 4 || rkn5_of(h->p) || lap_order_of(h->p) != 1 || ko_of(h->p) != 0)
      return fail(SH_EINVAL, "batched jobs must use the RK4 integrator, the 7-point Laplacian and no dissipation");
    if (h->capturing) return not_capturing(h);
    versions.push_back(h->layout_version);
    const Level& L = h->lev[0];
    const int off = (int)boxes.size();
    boxes.insert(boxes.end(), L.hbox.begin(), L.hbox.end());
    ctr.push_back(h->d_ls);
    std::vector<Tile> f, w, k;
    make_fused_tiles(L.boxes, b->tune, L.g.ng, f, batch_zc);
    if (!f.empty()) {
      for (Tile t : f) { t.box += off; ft.push_back(t); }
    } else {
      make_stage_tiles(L.boxes, b->tune, L.g.nvalid, w, k);
      for (Tile t : w) { t.box += off; wt.push_back(t); }
      for (Tile t : k) { t.box += off; bt.push_back(t); }
      std::vector<CopySeg> c;
      std::vector<long long> nc;
      build_a1(L, 1, c, nc);
      for (size_t i = 0; i < c.size(); ++i) {
        c[i].dbox += off;
        c[i].sbox += off;
        s1.push_back(c[i]);
        n1.push_back(nc[i]);
      }
    }
    std::vector<CopySeg> c;
    std::vector<long long> nc;
    build_a1(L, L.g.ng, c, nc);
    for (size_t i = 0; i < c.size(); ++i) {
      c[i].dbox += off;
      c[i].sbox += off;
      sd.push_back(c[i]);
      nd.push_back(nc[i]);
    }
  }
  const std::vector<SegBlock> b1 = wave_blocks(n1), bd = wave_blocks(nd);
  // byte sizes of the tables, in a fixed order
  struct Part {
    void** dev;
    size_t* n;
    size_t* cap;
    const void* src;
    size_t count, elem;
  };
  Part parts[] = {
      {(void**)&b->boxes.p, &b->boxes.n, &b->boxes.cap, boxes.data(), boxes.size(), sizeof(BoxDev)},
      {(void**)&b->ftiles.p, &b->ftiles.n, &b->ftiles.cap, ft.data(), ft.size(), sizeof(Tile)},
      {(void**)&b->wtiles.p, &b->wtiles.n, &b->wtiles.cap, wt.data(), wt.size(), sizeof(Tile)},
      {(void**)&b->btiles.p, &b->btiles.n, &b->btiles.cap, bt.data(), bt.size(), sizeof(Tile)},
      {(void**)&b->a1s_segs.p, &b->a1s_segs.n, &b->a1s_segs.cap, s1.data(), s1.size(), sizeof(CopySeg)},
      {(void**)&b->a1s_blocks.p, &b->a1s_blocks.n, &b->a1s_blocks.cap, b1.data(), b1.size(), sizeof(SegBlock)},
      {(void**)&b->a1d_segs.p, &b->a1d_segs.n, &b->a1d_segs.cap, sd.data(), sd.size(), sizeof(CopySeg)},
      {(void**)&b->a1d_blocks.p, &b->a1d_blocks.n, &b->a1d_blocks.cap, bd.data(), bd.size(), sizeof(SegBlock)},
      {(void**)&b->counters.p, &b->counters.n, &b->counters.cap, ctr.data(), ctr.size(), sizeof(LevelScal*)},
  };
  // grow the buffers that are too small (the stream must first finish with them)
  bool grow = false;
  size_t total = 0;
  for (const Part& q : parts) {
    grow = grow || q.count > *q.cap;
    total += (q.count * q.elem + 255) / 256 * 256;
  }
  if (grow) {
    HIPCHK(hipStreamSynchronize(b->st));
    for (const Part& q : parts)
      if (q.count > *q.cap) {
        if (*q.dev) (void)hipFree(*q.dev);
        *q.dev = nullptr;
        *q.cap = 0;
        const size_t c = std::max(q.count + q.count / 2, (size_t)64);
        HIPCHK(hipMalloc(q.dev, c * q.elem));
        *q.cap = c;
      }
  }
  // stage the contents in the next pinned buffer (waiting only if its last copies are
  // still queued) and copy them in stream order
  BatchStage& g = b->stage[b->next_stage];
  b->next_stage = (b->next_stage + 1) % SH_BATCH_STAGES;
  if (g.used) HIPCHK(hipEventSynchronize(g.done));
  if (g.cap < total) {
    if (g.buf) (void)hipHostFree(g.buf);
    g.buf = nullptr;
    g.cap = 0;
    const size_t c = std::max(total + total / 2, (size_t)1 << 16);
    HIPCHK(hipHostMalloc((void**)&g.buf, c, hipHostMallocDefault));
    g.cap = c;
  }
  if (!g.done) HIPCHK(hipEventCreateWithFlags(&g.done, hipEventDisableTiming));
  size_t o = 0;
  for (const Part& q : parts) {
    const size_t bytes = q.count * q.elem;
    *q.n = q.count;
    if (bytes) {
      std::memcpy(g.buf + o, q.src, bytes);
      HIPCHK(hipMemcpyAsync(*q.dev, g.buf + o, bytes, hipMemcpyHostToDevice, b->st));
    }
    o += (bytes + 255) / 256 * 256;
  }
  HIPCHK(hipEventRecord(g.done, b->st));
  g.used = true;
  b->jobs.assign(jobs, jobs + njobs);
  b->versions = versions;
  return SH_OK;
}

extern "C" {

sh_status sh_batch_create(int32_t njobs, const sh_hierarchy* jobs, sh_batch* out) {
  if (!out || njobs < 1 || !jobs || !jobs[0]) return fail(SH_EINVAL, "bad batch arguments");
  *out = nullptr;
  sh_batch b = new (std::nothrow) sh_batch_s;
  if (!b) return fail(SH_ENOMEM, "host allocation failed");
  b->st = jobs[0]->st;
  b->prec = jobs[0]->p.prec;
  b->tune = jobs[0]->tune;
  sh_status s = batch_set_jobs(b, njobs, jobs);
  if (s != SH_OK) {
    (void)hipStreamSynchronize(b->st);
    b->release();
    delete b;
    return s;
  }
  *out = b;
  return SH_OK;
}

sh_status sh_batch_update(sh_batch b, int32_t njobs, const sh_hierarchy* jobs) {
  if (!b || njobs < 1 || !jobs) return fail(SH_EINVAL, "bad batch arguments");
  return batch_set_jobs(b, njobs, jobs);
}

sh_status sh_batch_advance(sh_batch b) {
  if (!b) return fail(SH_EINVAL, "null batch");
  for (size_t j = 0; j < b->jobs.size(); ++j)
    if (b->jobs[j]->layout_version != b->versions[j]) return fail(SH_ESTATE, "a job's layout changed since batching");
  const int prec = b->prec;
  const bool nt = b->tune.nt != 0;
  if (b->ftiles.n) {
    sh_launch_fused(prec, nt, b->tune.fshape, b->tune.fvar, 4, b->ftiles.p, (int)b->ftiles.n, b->boxes.p, b->st);
    LAUNCHCHK();
  }
  if (b->wtiles.n || b->btiles.n) {
    const int role_in[4] = {ROLE_UN, ROLE_A, ROLE_B, ROLE_A};
    for (int s = 0; s < 4; ++s) {
      if (s > 0) {
        sh_launch_ghost_copy(prec, b->a1s_segs.p, b->a1s_blocks.p, (int)b->a1s_blocks.n, b->boxes.p,
                             role_in[s], 2, b->st);
        LAUNCHCHK();
      }
      if (b->btiles.n)
        sh_launch_stage(prec, s, b->tune.kind, nt, 1, 0, b->btiles.p, (int)b->btiles.n, b->boxes.p, b->st);
      if (b->wtiles.n) sh_launch_stage(prec, s, 0, nt, 1, 0, b->wtiles.p, (int)b->wtiles.n, b->boxes.p, b->st);
      LAUNCHCHK();
    }
  }
  sh_launch_counter_inc_list(b->counters.p, (int)b->counters.n, b->st);
  LAUNCHCHK();
  for (sh_hierarchy h : b->jobs) h->lev[0].k += 1;
  sh_launch_ghost_copy(prec, b->a1d_segs.p, b->a1d_blocks.p, (int)b->a1d_blocks.n, b->boxes.p, ROLE_UN, 4,
                       b->st);
  LAUNCHCHK();
  return SH_OK;
}

sh_status sh_batch_capture(sh_batch b, int32_t nsteps, sh_graph* out) {
  if (!b || !out || nsteps < 1) return fail(SH_EINVAL, "bad arguments");
  *out = nullptr;
  for (size_t j = 0; j < b->jobs.size(); ++j) {
    sh_status s = not_capturing(b->jobs[j]);
    if (s != SH_OK) return s;
    if (b->jobs[j]->layout_version != b->versions[j]) return fail(SH_ESTATE, "a job's layout changed since batching");
  }
  if (!b->st) return fail(SH_EINVAL, "the legacy default stream cannot be captured: create the jobs on a stream");
  HIPCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
  sh_status s = SH_OK;
  int recorded = 0;
  for (; recorded < nsteps && (s = sh_batch_advance(b)) == SH_OK; ++recorded) {
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->st, &g);
  for (sh_hierarchy h : b->jobs) h->lev[0].k -= recorded;  // recorded, not run
  if (s != SH_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return s != SH_OK ? s : fail(SH_EDEVICE, hipGetErrorString(e));
  }
  sh_graph G = new (std::nothrow) sh_graph_s;
  if (!G) {
    (void)hipGraphDestroy(g);
    return fail(SH_ENOMEM, "host allocation failed");
  }
  G->graph = g;
  G->st = b->st;
  for (size_t j = 0; j < b->jobs.size(); ++j) G->adv.push_back({b->jobs[j], 0, (long long)nsteps, b->versions[j]});
  e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    sh_graph_destroy(G);
    return fail(SH_EDEVICE, hipGetErrorString(e));
  }
  *out = G;
  return SH_OK;
}

sh_status sh_batch_destroy(sh_batch b) {
  if (!b) return SH_OK;
  (void)hipStreamSynchronize(b->st);
  b->release();
  delete b;
  return SH_OK;
}

}  // extern "C"
