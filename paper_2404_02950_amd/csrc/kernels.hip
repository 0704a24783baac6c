// HIP kernels of the per-level AMR time step for gfx950 (MI355X).
//
// Every kernel is gather-only: each output element has exactly one writer, and the only
// cross-thread combination is a fixed-shape reduction (energy) or a scan (tag
// compaction), so results do not depend on scheduling.  No fused multiply-add: the file
// is compiled with -ffp-contract=off and the pragma below repeats it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_internal.h"
#include "sh_launch.h"
#include "sh_device.h"
#include "sh_stage.h"

#pragma clang fp contract(off)

__global__ void k_counter_inc_list(LevelScal* const* ls, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ls[i]->k += 1;
}

__global__ void k_counter_inc(LevelScal* ls, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ls[i].k += 1;
}

__global__ void k_counter_zero(LevelScal* ls, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ls[i].k = 0;
}

// ---------------------------------------------------------------------------------
// A1: same-level ghost copy (periodic images included) of the first ncomp components:
// the psi pair on the stepping path, all four before a regrid interpolates from them.
// ---------------------------------------------------------------------------------
// One wavefront per chunk of up to 64 cells of a segment (four chunks per workgroup), so
// the many small edge and corner pieces of small boxes do not each take a workgroup.
template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_ghost_copy(const CopySeg* __restrict__ segs,
                                                         const SegBlock* __restrict__ chunks, int nchunks,
                                                         const BoxDev* __restrict__ boxes, int role, int ncomp) {
  const int ch = __builtin_amdgcn_readfirstlane(blockIdx.x * (SH_BLOCK / SH_WAVE) + (threadIdx.x >> 6));
  if (ch >= nchunks) return;  // uniform over the wavefront
  const SegBlock sb = chunks[ch];
  const CopySeg s = segs[sb.seg];
  const int c = sb.start + (threadIdx.x & (SH_WAVE - 1));
  if (c >= s.n[0] * s.n[1] * s.n[2]) return;
  const int i = c % s.n[0];
  const int r = c / s.n[0];
  const int j = r % s.n[1];
  const int k = r / s.n[1];
  const BoxDev& D = boxes[s.dbox];
  const BoxDev& Sb = boxes[s.sbox];
  const int sl = role_slot(role, load_level(D.ls));
  Glob<T>* dst = (Glob<T>*)D.slot[sl];
  const Glob<T>* src = (const Glob<T>*)Sb.slot[sl];
  const long long ed = elem<T>(D, s.dlo[0] + i, s.dlo[1] + j, s.dlo[2] + k);
  const long long es = elem<T>(Sb, s.slo[0] + i, s.slo[1] + j, s.slo[2] + k);
  for (int comp = 0; comp < ncomp; ++comp) dst[comp * D.cs + ed] = src[comp * Sb.cs + es];
}

// ---------------------------------------------------------------------------------
// A2: coarse->fine ghost interpolation of the psi components.  Time first:
//   C(alpha) = (1 - alpha) C_old + alpha C_new  (alpha = 0, 1: the stored state itself)
// then linear conservative space interpolation with central slopes (type 1):
//   f = ((C_I + t_x) + t_y) + t_z,  t_d = (C_{I+e_d} - C_{I-e_d}) * (+-1/8)
// or quartic conservative (type 4): the 1-D conservative quartic through the averages of
// the five coarse cells I-2..I+2, averaged over the child half-cell,
//   q(c) = c_0 + ((c_1 - c_-1) * (+-11/64) + (c_2 - c_-2) * (-+3/128)),
// applied along x for the 5 x 5 (y, z) neighbours, then along y, then along z.
// Arithmetic in float64, rounded to T on store.
// ---------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double tinterp(const Glob<T>* Cold, const Glob<T>* Cnew, long long e, int anum, double a) {
  if (anum == 4) return (double)Cnew[e];
  if (anum == 0) return (double)Cold[e];
  return (1.0 - a) * (double)Cold[e] + a * (double)Cnew[e];
}

// One workgroup per tile of parent cells of a segment (qtile_dims).  The time-interpolated
// coarse values of the tile grown by the reach G (1 linear, 2 quartic) go to LDS once per
// component, so every coarse value is read and time-interpolated once; each thread then
// forms all eight children of its parent, each child with the same operations in the same
// order as one child alone (quartic: the separable passes, x for both child parities on
// the 25 (y, z) rows, then y, then z), and stores those that lie in the segment's fine
// region.
template <typename T, int IT>
__global__ __launch_bounds__(SH_BLOCK) void k_ghost_interp(const InterpSeg* __restrict__ segs,
                                                             const SegBlock* __restrict__ blocks,
                                                             const BoxDev* __restrict__ fboxes,
                                                             const BoxDev* __restrict__ cboxes, int role,
                                                             int anum, int ncomp) {
  __shared__ double sm[QT_LDS];
  const SegBlock sb = blocks[blockIdx.x];
  const InterpSeg s = segs[sb.seg];
  const int tile = sb.start / SH_BLOCK;
  int p0[3], np[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    p0[d] = s.fg0[d] >> 1;  // floor: fine ghost indices may be negative
    np[d] = ((s.fg0[d] + s.n[d] - 1) >> 1) - p0[d] + 1;
  }
  int qt[3];
  qtile_dims(np, qt);
  const int ntx = (np[0] + qt[0] - 1) / qt[0], nty = (np[1] + qt[1] - 1) / qt[1];
  const int ix = tile % ntx, iy = (tile / ntx) % nty, iz = tile / (ntx * nty);
  const int t0[3] = {p0[0] + ix * qt[0], p0[1] + iy * qt[1], p0[2] + iz * qt[2]};
  const int tn[3] = {min(qt[0], np[0] - ix * qt[0]), min(qt[1], np[1] - iy * qt[1]), min(qt[2], np[2] - iz * qt[2])};
  constexpr int G = IT == 4 ? 2 : 1;
  const int sx = tn[0] + 2 * G, sy = tn[1] + 2 * G, sz = tn[2] + 2 * G;
  const BoxDev& F = fboxes[s.fbox];
  const BoxDev& C = cboxes[s.cbox];
  const LevelScal LC = load_level(C.ls);
  const Glob<T>* Cnew = (const Glob<T>*)C.slot[role_slot(ROLE_UN, LC)];
  const Glob<T>* Cold = (const Glob<T>*)C.slot[role_slot(ROLE_OLD, LC)];
  Glob<T>* dst = (Glob<T>*)F.slot[role_slot(role, load_level(F.ls))];
  const double a = 0.25 * (double)anum;
  const int tid = threadIdx.x;
  const bool has_p = tid < tn[0] * tn[1] * tn[2];
  const int pi = tid % tn[0], pj = (tid / tn[0]) % tn[1], pk = tid / (tn[0] * tn[1]);
  const double lo1 = -11.0 / 64.0, lo2 = 3.0 / 128.0, hi1 = 11.0 / 64.0, hi2 = -3.0 / 128.0;
  for (int comp = 0; comp < ncomp; ++comp) {
    const Glob<T>* co = Cold + comp * C.cs;
    const Glob<T>* cn = Cnew + comp * C.cs;
    for (int idx = tid; idx < sx * sy * sz; idx += SH_BLOCK) {
      const int u = idx % sx, v = (idx / sx) % sy, w = idx / (sx * sy);
      const long long e = elem<T>(C, t0[0] + u - G + s.cshift[0], t0[1] + v - G + s.cshift[1],
                                  t0[2] + w - G + s.cshift[2]);
      sm[idx] = tinterp(co, cn, e, anum, a);
    }
    __syncthreads();
    if (IT == 1 && has_p) {
      // linear: f = ((C + t_x) + t_y) + t_z, t_d = (C_{+d} - C_{-d}) * (+-1/8)
      const int c = ((pk + 1) * sy + (pj + 1)) * sx + pi + 1;
      const double c0 = sm[c];
      const double dx = sm[c + 1] - sm[c - 1], dy = sm[c + sx] - sm[c - sx], dz = sm[c + sx * sy] - sm[c - sx * sy];
#pragma unroll
      for (int zc = 0; zc < 2; ++zc)
#pragma unroll
        for (int yc = 0; yc < 2; ++yc)
#pragma unroll
          for (int xc = 0; xc < 2; ++xc) {
            const int fx = 2 * (t0[0] + pi) + xc, fy = 2 * (t0[1] + pj) + yc, fz = 2 * (t0[2] + pk) + zc;
            if (fx < s.fg0[0] || fx >= s.fg0[0] + s.n[0] || fy < s.fg0[1] || fy >= s.fg0[1] + s.n[1] ||
                fz < s.fg0[2] || fz >= s.fg0[2] + s.n[2])
              continue;
            const double tx = dx * (xc ? 0.125 : -0.125), ty = dy * (yc ? 0.125 : -0.125);
            const double tz = dz * (zc ? 0.125 : -0.125);
            const long long ed = elem<T>(F, s.flo[0] + fx - s.fg0[0], s.flo[1] + fy - s.fg0[1], s.flo[2] + fz - s.fg0[2]);
            dst[comp * F.cs + ed] = (T)(((c0 + tx) + ty) + tz);
          }
    }
    if (IT == 4 && has_p) {
      // one x child at a time (the 25 x-rows are read from LDS twice), which halves the
      // registers the separable passes hold; each child's operations are unchanged
#pragma unroll
      for (int xc = 0; xc < 2; ++xc) {
        const double a1 = xc ? hi1 : lo1, a2 = xc ? hi2 : lo2;
        double hz[2][5];  // [y child][z row]
#pragma unroll
        for (int dz = 0; dz < 5; ++dz) {
          double g[5];  // [y row]
#pragma unroll
          for (int dy = 0; dy < 5; ++dy) {
            const double* r = &sm[((pk + dz) * sy + (pj + dy)) * sx + pi];
            const double d1 = r[3] - r[1], d2 = r[4] - r[0];
            g[dy] = r[2] + (d1 * a1 + d2 * a2);
          }
          const double d1 = g[3] - g[1], d2 = g[4] - g[0];
          hz[0][dz] = g[2] + (d1 * lo1 + d2 * lo2);
          hz[1][dz] = g[2] + (d1 * hi1 + d2 * hi2);
        }
#pragma unroll
        for (int zc = 0; zc < 2; ++zc)
#pragma unroll
          for (int yc = 0; yc < 2; ++yc) {
            const int fx = 2 * (t0[0] + pi) + xc, fy = 2 * (t0[1] + pj) + yc, fz = 2 * (t0[2] + pk) + zc;
            if (fx < s.fg0[0] || fx >= s.fg0[0] + s.n[0] || fy < s.fg0[1] || fy >= s.fg0[1] + s.n[1] ||
                fz < s.fg0[2] || fz >= s.fg0[2] + s.n[2])
              continue;
            const double* h = hz[yc];
            const double d1 = h[3] - h[1], d2 = h[4] - h[0];
            const double val = h[2] + (zc ? (d1 * hi1 + d2 * hi2) : (d1 * lo1 + d2 * lo2));
            const long long ed = elem<T>(F, s.flo[0] + fx - s.fg0[0], s.flo[1] + fy - s.fg0[1], s.flo[2] + fz - s.fg0[2]);
            dst[comp * F.cs + ed] = (T)val;
          }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------
// A5: average down, all 4 components, fine U_n -> coarse U_n:
//   c = ((((f000+f100)+(f010+f110))+((f001+f101)+(f011+f111))) * 0.125)
// With tee: first the truncation error estimate |C - avg| (float64), stored on the 8
// children in the fine level's per-cell array: for tee_nc = 1 the maximum over the
// components (the first component's value unless a later one compares greater), for
// tee_nc = 4 each component's own (component c at tee + c * tee_cs).  write_coarse = 0
// keeps the coarse state (the shadow-level comparison).
// ---------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_avgdown(const AvgSeg* __restrict__ segs,
                                                      const SegBlock* __restrict__ blocks,
                                                      const BoxDev* __restrict__ cboxes,
                                                      const BoxDev* __restrict__ fboxes, double* __restrict__ tee,
                                                      int tee_nc, long long tee_cs, int write_coarse) {
  const SegBlock sb = blocks[blockIdx.x];
  const AvgSeg s = segs[sb.seg];
  const int c = sb.start + threadIdx.x;
  if (c >= s.n[0] * s.n[1] * s.n[2]) return;
  const int i = c % s.n[0];
  const int r = c / s.n[0];
  const int j = r % s.n[1];
  const int k = r / s.n[1];
  const BoxDev& C = cboxes[s.cbox];
  const BoxDev& F = fboxes[s.fbox];
  Glob<T>* dst = (Glob<T>*)slot_base(C, role_slot(ROLE_UN, load_level(C.ls)));
  const Glob<T>* src = (const Glob<T>*)slot_base(F, role_slot(ROLE_UN, load_level(F.ls)));
  const long long ec = elem<T>(C, s.clo[0] + i, s.clo[1] + j, s.clo[2] + k);
  const long long ef = elem<T>(F, s.f0[0] + 2 * i, s.f0[1] + 2 * j, s.f0[2] + 2 * k);
  const long long px = F.px, plane = px * F.py;
  double t = 0.0, dc[4];
  for (int comp = 0; comp < 4; ++comp) {
    const Glob<T>* f = src + comp * F.cs + ef;
    const double f000 = f[0], f100 = f[1], f010 = f[px], f110 = f[px + 1];
    const double f001 = f[plane], f101 = f[plane + 1], f011 = f[plane + px], f111 = f[plane + px + 1];
    const double avg = ((((f000 + f100) + (f010 + f110)) + ((f001 + f101) + (f011 + f111))) * 0.125);
    if (tee) {
      const double d = fabs((double)dst[comp * C.cs + ec] - avg);
      dc[comp] = d;
      t = (comp == 0 || d > t) ? d : t;
    }
    if (write_coarse) dst[comp * C.cs + ec] = (T)avg;
  }
  if (tee) {
    const int x0 = s.f0[0] + 2 * i, y0 = s.f0[1] + 2 * j, z0 = s.f0[2] + 2 * k;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy) {
        const long long row = F.mask_off + ((long long)(z0 + dz) * F.ny + (y0 + dy)) * F.nx + x0;
        if (tee_nc == 4) {
          for (int comp = 0; comp < 4; ++comp) {
            tee[comp * tee_cs + row] = dc[comp];
            tee[comp * tee_cs + row + 1] = dc[comp];
          }
        } else {
          tee[row] = t;
          tee[row + 1] = t;
        }
      }
  }
}

// ---------------------------------------------------------------------------------
// Debug: NaN into the ghost shell (ng cells deep, the first ncomp components) of buffer
// `role` of every box of a level, before a fill that is meant to set all of it; a ghost
// cell a stencil reads but no fill writes then turns valid cells into NaN.  One block per
// (box, plane of the padded box).
// ---------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_poison_ghosts(const BoxDev* __restrict__ boxes, int nplanes, int ng,
                                                            int role, int ncomp) {
  const int b = blockIdx.x / nplanes;
  const int z = (int)(blockIdx.x % nplanes) - ng;
  const BoxDev B = boxes[b];
  if (z >= B.nz + ng) return;
  T* U = (T*)slot_base(B, role_slot(role, *B.ls));
  const T nan = __builtin_nan("");
  const int wx = B.nx + 2 * ng, wy = B.ny + 2 * ng;
  const bool zin = z >= 0 && z < B.nz;
  for (int q = threadIdx.x; q < wx * wy; q += SH_BLOCK) {
    const int x = q % wx - ng, y = q / wx - ng;
    if (zin && x >= 0 && x < B.nx && y >= 0 && y < B.ny) continue;
    const long long e = elem<T>(B, x, y, z);
    for (int c = 0; c < ncomp; ++c) U[c * B.cs + e] = nan;
  }
}

// Regrid: copy the 4 components of valid cells from the old layout of a level.
template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_regrid_copy(const CopySeg* __restrict__ segs,
                                                          const SegBlock* __restrict__ blocks,
                                                          const BoxDev* __restrict__ dboxes,
                                                          const BoxDev* __restrict__ sboxes,
                                                          const double* __restrict__ tee_src,
                                                          double* __restrict__ tee_dst, int tee_nc,
                                                          long long tee_cs_src, long long tee_cs_dst) {
  const SegBlock sb = blocks[blockIdx.x];
  const CopySeg s = segs[sb.seg];
  const int c = sb.start + threadIdx.x;
  if (c >= s.n[0] * s.n[1] * s.n[2]) return;
  const int i = c % s.n[0];
  const int r = c / s.n[0];
  const int j = r % s.n[1];
  const int k = r / s.n[1];
  const BoxDev& D = dboxes[s.dbox];
  const BoxDev& Sb = sboxes[s.sbox];
  T* dst = (T*)D.slot[role_slot(ROLE_UN, *D.ls)];
  const T* src = (const T*)Sb.slot[role_slot(ROLE_UN, *Sb.ls)];
  const long long ed = elem<T>(D, s.dlo[0] + i, s.dlo[1] + j, s.dlo[2] + k);
  const long long es = elem<T>(Sb, s.slo[0] + i, s.slo[1] + j, s.slo[2] + k);
  for (int comp = 0; comp < 4; ++comp) dst[comp * D.cs + ed] = src[comp * Sb.cs + es];
  // the truncation error estimate of a kept cell stays with it
  if (tee_src) {
    const long long cd = D.mask_off + ((long long)(s.dlo[2] + k) * D.ny + (s.dlo[1] + j)) * D.nx + (s.dlo[0] + i);
    const long long cs = Sb.mask_off + ((long long)(s.slo[2] + k) * Sb.ny + (s.slo[1] + j)) * Sb.nx + (s.slo[0] + i);
    for (int comp = 0; comp < tee_nc; ++comp) tee_dst[comp * tee_cs_dst + cd] = tee_src[comp * tee_cs_src + cs];
  }
}

// ---------------------------------------------------------------------------------
// A4: plaquette tagging.  W = sum over the 4 directed edges p->q of
//   +1 if y_p <= 0 < y_q and x_p y_q - x_q y_p > 0
//   -1 if y_q <= 0 < y_p and x_p y_q - x_q y_p < 0
// (crossing rule for the origin, D. Sunday 2001), in float64.  A cell is tagged iff any
// of its 12 incident plaquettes has W != 0.  Writes the byte mask of valid cells and a
// per-tile count (wave ballots).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ int edge_w(double xp, double yp, double xq, double yq) {
  const double cr = xp * yq - xq * yp;
  const int up = (yp <= 0.0) && (yq > 0.0) && (cr > 0.0);
  const int dn = (yq <= 0.0) && (yp > 0.0) && (cr < 0.0);
  return up - dn;
}

__device__ __forceinline__ bool pierced(const double* X, const double* Y, int a, int b, int c, int d) {
  // corners v0=a, v1=b, v2=c, v3=d
  const int w = edge_w(X[a], Y[a], X[b], Y[b]) + edge_w(X[b], Y[b], X[c], Y[c]) +
                edge_w(X[c], Y[c], X[d], Y[d]) + edge_w(X[d], Y[d], X[a], Y[a]);
  return w != 0;
}

template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_tag(const Tile* __restrict__ tiles, int ntiles,
                                                  const BoxDev* __restrict__ boxes, uint8_t* __restrict__ mask,
                                                  int* __restrict__ tile_count, const double* __restrict__ tee,
                                                  const TeeSpec te, int mode) {
  const int lane = threadIdx.x & (SH_WAVE - 1);
  const int t = blockIdx.x * (SH_BLOCK / SH_WAVE) + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const Tile tl = tiles[t];
  if (tl.box < 0) {
    if (lane == 0) tile_count[t] = 0;
    return;
  }
  const BoxDev B = boxes[tl.box];
  const T* __restrict__ U = (const T*)slot_base(B, role_slot(ROLE_UN, *B.ls));
  const int tx = lane & ((1 << tl.txs) - 1), ty = lane >> tl.txs;
  int x = (tl.xy & 0xffff) + tx, y = (tl.xy >> 16) + ty;
  const bool active = (x < B.nx) && (y < B.ny);
  x = min(x, B.nx - 1);
  y = min(y, B.ny - 1);
  const int z0 = tl.zz & 0xffff, zend = min(z0 + (tl.zz >> 16), B.nz);
  const long long px = B.px, plane = px * B.py, cs = B.cs;
  int count = 0;
  for (int z = z0; z < zend; ++z) {
    const long long cell = B.mask_off + ((long long)z * B.ny + y) * B.nx + x;
    bool tag = false;
    if (mode & 2) {
      if (te.nc == 4) {
#pragma unroll
        for (int c = 0; c < 4; ++c) tag = tag || (te.scale[c] * tee[c * te.cs + cell] > te.crit[c]);
      } else {
        tag = tee[cell] > te.crit[0];
      }
    }
    if (!(mode & 1)) {
      tag = tag && active;
      if (active) mask[cell] = tag ? 1 : 0;
      count += __popcll(__ballot(tag));
      continue;
    }
    const long long e = elem<T>(B, x, y, z);
    // 3x3x3 neighbourhood, index (dz+1)*9 + (dy+1)*3 + (dx+1); corners unused
    double X[27], Y[27];
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int id = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
          if (dx != 0 && dy != 0 && dz != 0) {
            X[id] = 0.0;
            Y[id] = 0.0;
            continue;
          }
          const long long o = e + dz * plane + dy * px + dx;
          X[id] = (double)U[o];
          Y[id] = (double)U[cs + o];
        }
#define ID(dx, dy, dz) (((dz) + 1) * 9 + ((dy) + 1) * 3 + ((dx) + 1))
    // normal z, axes (x, y): lower corners (x-1..x, y-1..y) in plane z
#pragma unroll
    for (int cy = -1; cy <= 0; ++cy)
#pragma unroll
      for (int cx = -1; cx <= 0; ++cx)
        tag |= pierced(X, Y, ID(cx, cy, 0), ID(cx + 1, cy, 0), ID(cx + 1, cy + 1, 0), ID(cx, cy + 1, 0));
    // normal x, axes (y, z): lower corners (y-1..y, z-1..z) in plane x
#pragma unroll
    for (int cz = -1; cz <= 0; ++cz)
#pragma unroll
      for (int cy = -1; cy <= 0; ++cy)
        tag |= pierced(X, Y, ID(0, cy, cz), ID(0, cy + 1, cz), ID(0, cy + 1, cz + 1), ID(0, cy, cz + 1));
    // normal y, axes (z, x): lower corners (z-1..z, x-1..x) in plane y
#pragma unroll
    for (int cx = -1; cx <= 0; ++cx)
#pragma unroll
      for (int cz = -1; cz <= 0; ++cz)
        tag |= pierced(X, Y, ID(cx, 0, cz), ID(cx, 0, cz + 1), ID(cx + 1, 0, cz + 1), ID(cx + 1, 0, cz));
#undef ID
    tag = tag && active;
    if (active) mask[cell] = tag ? 1 : 0;
    count += __popcll(__ballot(tag));
  }
  if (lane == 0) tile_count[t] = count;
}

// Exclusive scan of the per-tile counts (one block; sequential over chunks).
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ in, long long* __restrict__ out, int n) {
  __shared__ long long part[1024];
  const int tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b = tid * per, e = min(n, b + per);
  long long s = 0;
  for (int i = b; i < e; ++i) s += in[i];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    long long run = 0;
    for (int i = 0; i < 1024; ++i) {
      const long long v = part[i];
      part[i] = run;
      run += v;
    }
    out[n] = run;
  }
  __syncthreads();
  long long run = part[tid];
  for (int i = b; i < e; ++i) {
    out[i] = run;
    run += in[i];
  }
}

// Compaction of tagged cells to global (x, y, z) triplets in tile order.
__global__ __launch_bounds__(SH_BLOCK) void k_tag_compact(const Tile* __restrict__ tiles, int ntiles,
                                                          const BoxDev* __restrict__ boxes,
                                                          const uint8_t* __restrict__ mask,
                                                          const long long* __restrict__ tile_off,
                                                          int* __restrict__ idx, long long cap) {
  const int lane = threadIdx.x & (SH_WAVE - 1);
  const int t = blockIdx.x * (SH_BLOCK / SH_WAVE) + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const Tile tl = tiles[t];
  if (tl.box < 0) return;
  const BoxDev B = boxes[tl.box];
  const int tx = lane & ((1 << tl.txs) - 1), ty = lane >> tl.txs;
  const int x = (tl.xy & 0xffff) + tx, y = (tl.xy >> 16) + ty;
  const bool active = (x < B.nx) && (y < B.ny);
  const int z0 = tl.zz & 0xffff, zend = min(z0 + (tl.zz >> 16), B.nz);
  long long pos = tile_off[t];
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int z = z0; z < zend; ++z) {
    const bool tag = active && mask[B.mask_off + ((long long)z * B.ny + y) * B.nx + x];
    const unsigned long long bal = __ballot(tag);
    if (tag) {
      const long long p = pos + __popcll(bal & below);
      if (p < cap) {
        idx[3 * p + 0] = B.lo[0] + x;
        idx[3 * p + 1] = B.lo[1] + y;
        idx[3 * p + 2] = B.lo[2] + z;
      }
    }
    pos += __popcll(bal);
  }
}

// Tagged blocks for clustering, without a tag list: every tagged cell c (its parent c / 2
// when `halve`) sets, in the bitsets of the octants its cube [c - r, c + r] reaches, the
// bit of its own block B = c / b (b = 2^bsh cells; b/2 <= r < b, so along each axis the
// cube meets B and B - 1 when c's offset in B is < r, B + 1 when offset + r >= b, or both).
// The host grows each octant bitset by one block towards its octant.  Bit k = x + nb (y +
// nb z) of B lies in word k / 64 of octant o's nwords words.  Lanes with the same word
// are ORed together first, and one lane per word does the atomic.
__global__ __launch_bounds__(SH_BLOCK) void k_tag_octants(const Tile* __restrict__ tiles, int ntiles,
                                                          const BoxDev* __restrict__ boxes,
                                                          const uint8_t* __restrict__ mask, int halve, int r,
                                                          int bsh, int nb, unsigned long long* __restrict__ oct,
                                                          long long nwords) {
  const int lane = threadIdx.x & (SH_WAVE - 1);
  const int t = blockIdx.x * (SH_BLOCK / SH_WAVE) + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const Tile tl = tiles[t];
  if (tl.box < 0) return;
  const BoxDev B = boxes[tl.box];
  const int tx = lane & ((1 << tl.txs) - 1), ty = lane >> tl.txs;
  const int x = (tl.xy & 0xffff) + tx, y = (tl.xy >> 16) + ty;
  const bool active = (x < B.nx) && (y < B.ny);
  const int z0 = tl.zz & 0xffff, zend = min(z0 + (tl.zz >> 16), B.nz);
  const int b = 1 << bsh;
  const int cx = (B.lo[0] + x) >> halve, cy = (B.lo[1] + y) >> halve;
  const int ox = ((cx & (b - 1)) < r ? 1 : 0) | ((cx & (b - 1)) + r >= b ? 2 : 0);
  const int oy = ((cy & (b - 1)) < r ? 1 : 0) | ((cy & (b - 1)) + r >= b ? 2 : 0);
  for (int z = z0; z < zend; ++z) {
    const bool tag = active && mask[B.mask_off + ((long long)z * B.ny + y) * B.nx + x];
    if (!__ballot(tag)) continue;
    const int cz = (B.lo[2] + z) >> halve;
    const int oz = ((cz & (b - 1)) < r ? 1 : 0) | ((cz & (b - 1)) + r >= b ? 2 : 0);
    const long long k = ((long long)(cz >> bsh) * nb + (cy >> bsh)) * nb + (cx >> bsh);
    const unsigned long long bit = 1ull << (k & 63);
    // octant index: bit 0 set for +x, bit 1 for +y, bit 2 for +z
    for (int o = 0; o < 8; ++o) {
      const bool want = tag && ((o & 1) ? (ox & 2) : (ox & 1)) && ((o & 2) ? (oy & 2) : (oy & 1)) &&
                        ((o & 4) ? (oz & 2) : (oz & 1));
      const long long key = want ? (long long)o * nwords + (k >> 6) : -1;
      unsigned long long pending = __ballot(want);
      while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const long long lk = __shfl(key, leader);
        const bool mine = want && key == lk;
        unsigned long long v = mine ? bit : 0ull;
        for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off);
        if (lane == leader) atomicOr(oct + lk, v);
        pending &= ~__ballot(mine);
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// A6: energy.  Per cell (not covered by a finer level):
//   kin = 1/2 (Pi1^2 + Pi2^2),  grad = 1/2 sum_i sum_d (psi_i(x+e_d) - psi_i(x))^2 inv_dx2,
//   pot = 1/4 c_pot (r2 - 1)^2
// summed per lane over z, then over the wave by a fixed xor tree, one partial per tile.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_energy(const Tile* __restrict__ tiles, int ntiles,
                                                     const BoxDev* __restrict__ boxes,
                                                     const uint8_t* __restrict__ covered,
                                                     EnergyPartial* __restrict__ part) {
  const int lane = threadIdx.x & (SH_WAVE - 1);
  const int t = blockIdx.x * (SH_BLOCK / SH_WAVE) + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const Tile tl = tiles[t];
  double kin = 0.0, grad = 0.0, pot = 0.0;
  long long bad = 0;
  if (tl.box >= 0) {
    const BoxDev B = boxes[tl.box];
    const LevelScal L = *B.ls;
    const double cp = L.lam * ipow(level_time(L), L.beta);
    const T* __restrict__ U = (const T*)slot_base(B, role_slot(ROLE_UN, L));
    const int tx = lane & ((1 << tl.txs) - 1), ty = lane >> tl.txs;
    const int x = (tl.xy & 0xffff) + tx, y = (tl.xy >> 16) + ty;
    if (x < B.nx && y < B.ny) {
      const int z0 = tl.zz & 0xffff, zend = min(z0 + (tl.zz >> 16), B.nz);
      const long long px = B.px, plane = px * B.py, cs = B.cs;
      for (int z = z0; z < zend; ++z) {
        if (covered && covered[B.mask_off + ((long long)z * B.ny + y) * B.nx + x]) continue;
        const long long e = elem<T>(B, x, y, z);
        const double p1 = U[e], p2 = U[cs + e], q1 = U[2 * cs + e], q2 = U[3 * cs + e];
        kin += 0.5 * (q1 * q1 + q2 * q2);
        double g = 0.0;
        for (int c = 0; c < 2; ++c) {
          const T* u = U + c * cs;
          const double v = u[e];
          const double dxv = (double)u[e + 1] - v, dyv = (double)u[e + px] - v, dzv = (double)u[e + plane] - v;
          g = g + dxv * dxv;
          g = g + dyv * dyv;
          g = g + dzv * dzv;
        }
        grad += 0.5 * g * L.inv_dx2;
        const double r2m1 = (p1 * p1 + p2 * p2) - 1.0;
        pot += 0.25 * cp * (r2m1 * r2m1);
        bad += !(isfinite(p1) && isfinite(p2) && isfinite(q1) && isfinite(q2));
      }
    }
  }
  kin = wave_sum(kin);
  grad = wave_sum(grad);
  pot = wave_sum(pot);
  const double badd = wave_sum((double)bad);
  if (lane == 0) {
    part[t].kin = kin;
    part[t].grad = grad;
    part[t].pot = pot;
    part[t].nonfinite = (long long)badd;
  }
}

// Largest |U_c| per component over the valid cells of each tile (the maxima appendix D
// normalises truncation error estimates by).  A NaN anywhere makes the maximum NaN.
__device__ __forceinline__ double nanmax(double m, double v) { return (v > m || v != v) ? v : m; }

__device__ __forceinline__ double wave_nanmax(double v) {
#pragma unroll
  for (int o = SH_WAVE / 2; o >= 1; o >>= 1) v = nanmax(v, __shfl_xor(v, o));
  return v;
}

template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_absmax(const Tile* __restrict__ tiles, int ntiles,
                                                     const BoxDev* __restrict__ boxes, double* __restrict__ part) {
  const int lane = threadIdx.x & (SH_WAVE - 1);
  const int t = blockIdx.x * (SH_BLOCK / SH_WAVE) + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const Tile tl = tiles[t];
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  if (tl.box >= 0) {
    const BoxDev B = boxes[tl.box];
    const T* __restrict__ U = (const T*)slot_base(B, role_slot(ROLE_UN, *B.ls));
    const int tx = lane & ((1 << tl.txs) - 1), ty = lane >> tl.txs;
    const int x = (tl.xy & 0xffff) + tx, y = (tl.xy >> 16) + ty;
    if (x < B.nx && y < B.ny) {
      const int z0 = tl.zz & 0xffff, zend = min(z0 + (tl.zz >> 16), B.nz);
      for (int z = z0; z < zend; ++z) {
        const long long e = elem<T>(B, x, y, z);
#pragma unroll
        for (int c = 0; c < 4; ++c) m[c] = nanmax(m[c], fabs((double)U[c * B.cs + e]));
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) m[c] = wave_nanmax(m[c]);
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) part[4 * (long long)t + c] = m[c];
}

// Maximum over the per-tile partials (one block), per component.
__global__ __launch_bounds__(256) void k_absmax_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sm[4][256];
  const int tid = threadIdx.x;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = tid; i < n; i += 256)
#pragma unroll
    for (int c = 0; c < 4; ++c) m[c] = nanmax(m[c], part[4 * (long long)i + c]);
#pragma unroll
  for (int c = 0; c < 4; ++c) sm[c][tid] = m[c];
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o)
#pragma unroll
      for (int c = 0; c < 4; ++c) sm[c][tid] = nanmax(sm[c][tid], sm[c][tid + o]);
    __syncthreads();
  }
  if (tid < 4) out[tid] = sm[tid][0];
}

// Fixed-order final sum of the per-tile partials (one block): out = [kin, grad, pot, nonfinite].
__global__ __launch_bounds__(256) void k_energy_final(const EnergyPartial* __restrict__ part, int n,
                                                      double vol, double* __restrict__ out) {
  __shared__ double sk[256], sg[256], sp[256], sb[256];
  const int tid = threadIdx.x;
  double k = 0.0, g = 0.0, p = 0.0, b = 0.0;
  for (int i = tid; i < n; i += 256) {
    k += part[i].kin;
    g += part[i].grad;
    p += part[i].pot;
    b += (double)part[i].nonfinite;
  }
  sk[tid] = k; sg[tid] = g; sp[tid] = p; sb[tid] = b;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) {
      sk[tid] += sk[tid + o];
      sg[tid] += sg[tid + o];
      sp[tid] += sp[tid + o];
      sb[tid] += sb[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = sk[0] * vol;
    out[1] = sg[0] * vol;
    out[2] = sp[0] * vol;
    out[3] = sb[0];
  }
}

// Mark coarse cells covered by a finer level (for the composite energy).
__global__ __launch_bounds__(SH_BLOCK) void k_mark_covered(const AvgSeg* __restrict__ segs,
                                                           const SegBlock* __restrict__ blocks,
                                                           const BoxDev* __restrict__ cboxes,
                                                           uint8_t* __restrict__ covered) {
  const SegBlock sb = blocks[blockIdx.x];
  const AvgSeg s = segs[sb.seg];
  const int c = sb.start + threadIdx.x;
  if (c >= s.n[0] * s.n[1] * s.n[2]) return;
  const int i = c % s.n[0];
  const int r = c / s.n[0];
  const int j = r % s.n[1];
  const int k = r / s.n[1];
  const BoxDev& C = cboxes[s.cbox];
  covered[C.mask_off + ((long long)(s.clo[2] + k) * C.ny + (s.clo[1] + j)) * C.nx + (s.clo[0] + i)] = 1;
}

// ---------------------------------------------------------------------------------
// State transfer between box storage and a dense float64 staging buffer laid out as
// [box][comp][z][y][x] (valid cells, or with the ghost shell when g = 1).
// ---------------------------------------------------------------------------------
template <typename T, bool TO_BOX>
__global__ __launch_bounds__(SH_BLOCK) void k_xfer(const BoxDev* __restrict__ boxes, const long long* __restrict__ off,
                                                   int nbox, double* __restrict__ stage, int role, int g,
                                                   long long total) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  // find the box by binary search over off[0..nbox]
  int lo = 0, hi = nbox;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= gid) lo = mid; else hi = mid;
  }
  const BoxDev& B = boxes[lo];
  const int ex = B.nx + 2 * g, ey = B.ny + 2 * g, ez = B.nz + 2 * g;
  long long r = gid - off[lo];
  const long long per = (long long)ex * ey * ez;
  const int comp = (int)(r / per);
  r -= comp * per;
  const int i = (int)(r % ex) - g;
  const int j = (int)((r / ex) % ey) - g;
  const int k = (int)(r / ((long long)ex * ey)) - g;
  T* S = (T*)slot_base(B, role_slot(role, *B.ls));
  const long long e = comp * B.cs + elem<T>(B, i, j, k);
  if (TO_BOX) S[e] = (T)stage[gid];
  else stage[gid] = (double)S[e];
}

// ---------------------------------------------------------------------------------
// Launch wrappers (host side).
// ---------------------------------------------------------------------------------
static inline int nblk(long long n, int per) { return (int)((n + per - 1) / per); }

// kind: 0 = wave-row tiles (k_stage), 4 or 8 = block-row tiles of that many rows;
// order: the Laplacian order (1 here, 2 and 3 in kernels_hilap.hip); ko: dissipation
// order (kernels_ko.hip)
void sh_launch_stage(int prec, int s, int kind, bool nt, int order, int ko, const Tile* tiles, int ntiles,
                     const BoxDev* boxes, hipStream_t st) {
  if (ko > 0 && kind != 0) sh_launch_stage_ko_lds(prec, s, kind, nt, order, ko, tiles, ntiles, boxes, st);
  else if (ko > 0) sh_launch_stage_ko(prec, s, nt, order, ko, tiles, ntiles, boxes, st);
  else if (order > 1) sh_launch_stage_hilap(prec, s, kind, nt, order, tiles, ntiles, boxes, st);
  else stage_launch_radius<1>(prec, s, kind, nt, tiles, ntiles, boxes, st);
}

void sh_launch_rhs(int prec, int order, int ko, const Tile* tiles, int ntiles, const BoxDev* boxes,
                   const long long* out_off, double* out, hipStream_t st) {
  if (ko > 0) sh_launch_rhs_ko(prec, order, ko, tiles, ntiles, boxes, out_off, out, st);
  else if (order > 1) sh_launch_rhs_hilap(prec, order, tiles, ntiles, boxes, out_off, out, st);
  else rhs_launch_radius<1>(prec, tiles, ntiles, boxes, out_off, out, st);
}

void sh_launch_counter_inc_list(LevelScal* const* ls, int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_counter_inc_list, dim3(nblk(n, 64)), dim3(64), 0, st, ls, n);
}

void sh_launch_counter_inc(LevelScal* ls, int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_counter_inc, dim3(nblk(n, 64)), dim3(64), 0, st, ls, n);
}

void sh_launch_ghost_copy(int prec, const CopySeg* segs, const SegBlock* chunks, int nchunks, const BoxDev* boxes,
                          int role, int ncomp, hipStream_t st) {
  if (nchunks == 0) return;
  const int per = SH_BLOCK / SH_WAVE;
  const dim3 grid((nchunks + per - 1) / per);
  if (prec == 0)
    hipLaunchKernelGGL(k_ghost_copy<double>, grid, dim3(SH_BLOCK), 0, st, segs, chunks, nchunks, boxes, role, ncomp);
  else
    hipLaunchKernelGGL(k_ghost_copy<float>, grid, dim3(SH_BLOCK), 0, st, segs, chunks, nchunks, boxes, role, ncomp);
}

// the plan's blocks are parent tiles (qtile_dims)
template <int IT>
static void ghost_interp_launch(int prec, const InterpSeg* segs, const SegBlock* blocks, int nblocks,
                                const BoxDev* fboxes, const BoxDev* cboxes, int role, int anum, int ncomp,
                                hipStream_t st) {
  if (prec == 0)
    hipLaunchKernelGGL((k_ghost_interp<double, IT>), dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, fboxes,
                       cboxes, role, anum, ncomp);
  else
    hipLaunchKernelGGL((k_ghost_interp<float, IT>), dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, fboxes, cboxes,
                       role, anum, ncomp);
}

void sh_launch_ghost_interp(int prec, int interp, const InterpSeg* segs, const SegBlock* blocks, int nblocks,
                            const BoxDev* fboxes, const BoxDev* cboxes, int role, int anum, int ncomp,
                            hipStream_t st) {
  if (nblocks == 0) return;
  if (interp == 4) ghost_interp_launch<4>(prec, segs, blocks, nblocks, fboxes, cboxes, role, anum, ncomp, st);
  else ghost_interp_launch<1>(prec, segs, blocks, nblocks, fboxes, cboxes, role, anum, ncomp, st);
}

void sh_launch_avgdown(int prec, const AvgSeg* segs, const SegBlock* blocks, int nblocks, const BoxDev* cboxes,
                       const BoxDev* fboxes, double* tee, int tee_nc, long long tee_cs, int write_coarse,
                       hipStream_t st) {
  if (nblocks == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL(k_avgdown<double>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, cboxes, fboxes, tee,
                       tee_nc, tee_cs, write_coarse);
  else
    hipLaunchKernelGGL(k_avgdown<float>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, cboxes, fboxes, tee,
                       tee_nc, tee_cs, write_coarse);
}

void sh_launch_regrid_copy(int prec, const CopySeg* segs, const SegBlock* blocks, int nblocks, const BoxDev* dboxes,
                           const BoxDev* sboxes, const double* tee_src, double* tee_dst, int tee_nc,
                           long long tee_cs_src, long long tee_cs_dst, hipStream_t st) {
  if (nblocks == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL(k_regrid_copy<double>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, dboxes, sboxes,
                       tee_src, tee_dst, tee_nc, tee_cs_src, tee_cs_dst);
  else
    hipLaunchKernelGGL(k_regrid_copy<float>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, dboxes, sboxes,
                       tee_src, tee_dst, tee_nc, tee_cs_src, tee_cs_dst);
}

void sh_launch_tag(int prec, const Tile* tiles, int ntiles, const BoxDev* boxes, uint8_t* mask, int* tile_count,
                   const double* tee, const TeeSpec& te, int mode, hipStream_t st) {
  const int nb = nblk(ntiles, SH_BLOCK / SH_WAVE);
  if (nb == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL(k_tag<double>, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, mask, tile_count, tee,
                       te, mode);
  else
    hipLaunchKernelGGL(k_tag<float>, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, mask, tile_count, tee,
                       te, mode);
}

void sh_launch_scan(const int* in, long long* out, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, in, out, n);
}

void sh_launch_tag_compact(const Tile* tiles, int ntiles, const BoxDev* boxes, const uint8_t* mask,
                           const long long* tile_off, int* idx, long long cap, hipStream_t st) {
  const int nb = nblk(ntiles, SH_BLOCK / SH_WAVE);
  if (nb == 0) return;
  hipLaunchKernelGGL(k_tag_compact, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, mask, tile_off, idx, cap);
}

void sh_launch_tag_octants(const Tile* tiles, int ntiles, const BoxDev* boxes, const uint8_t* mask, int halve, int r,
                           int bsh, int nb, unsigned long long* oct, long long nwords, hipStream_t st) {
  const int n = nblk(ntiles, SH_BLOCK / SH_WAVE);
  if (n == 0) return;
  hipLaunchKernelGGL(k_tag_octants, dim3(n), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, mask, halve, r, bsh, nb, oct,
                     nwords);
}

void sh_launch_energy(int prec, const Tile* tiles, int ntiles, const BoxDev* boxes, const uint8_t* covered,
                      EnergyPartial* part, hipStream_t st) {
  const int nb = nblk(ntiles, SH_BLOCK / SH_WAVE);
  if (nb == 0) return;
  if (prec == 0) hipLaunchKernelGGL(k_energy<double>, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, covered, part);
  else hipLaunchKernelGGL(k_energy<float>, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, covered, part);
}

void sh_launch_energy_final(const EnergyPartial* part, int n, double vol, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, st, part, n, vol, out);
}

void sh_launch_mark_covered(const AvgSeg* segs, const SegBlock* blocks, int nblocks, const BoxDev* cboxes,
                            uint8_t* covered, hipStream_t st) {
  if (nblocks == 0) return;
  hipLaunchKernelGGL(k_mark_covered, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, cboxes, covered);
}

void sh_launch_xfer(int prec, bool to_box, const BoxDev* boxes, const long long* off, int nbox, double* stage, int role,
                    int g, long long total, hipStream_t st) {
  if (total == 0) return;
  const int nb = nblk(total, SH_BLOCK);
  if (prec == 0) {
    if (to_box) hipLaunchKernelGGL((k_xfer<double, true>), dim3(nb), dim3(SH_BLOCK), 0, st, boxes, off, nbox, stage, role, g, total);
    else hipLaunchKernelGGL((k_xfer<double, false>), dim3(nb), dim3(SH_BLOCK), 0, st, boxes, off, nbox, stage, role, g, total);
  } else {
    if (to_box) hipLaunchKernelGGL((k_xfer<float, true>), dim3(nb), dim3(SH_BLOCK), 0, st, boxes, off, nbox, stage, role, g, total);
    else hipLaunchKernelGGL((k_xfer<float, false>), dim3(nb), dim3(SH_BLOCK), 0, st, boxes, off, nbox, stage, role, g, total);
  }
}

// Diagnostic: the stage scalars the device derives (for bitwise checks against the host).
__global__ void k_debug_scalars(const LevelScal* ls, int s, double* out) {
  const LevelScal L = *ls;
  const StageScal sc = stage_scalars(L, s);
  out[0] = level_time(L) + stage_frac(s) * L.dt;
  out[1] = sc.cf;
  out[2] = sc.cp;
  out[3] = sc.h6;
  out[4] = sc.h3;
  out[5] = sc.h2;
  out[6] = sc.h1;
}

void sh_launch_debug_scalars(const LevelScal* ls, int s, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_debug_scalars, dim3(1), dim3(1), 0, st, ls, s, out);
}

void sh_launch_absmax(int prec, const Tile* tiles, int ntiles, const BoxDev* boxes, double* part, double* out,
                      hipStream_t st) {
  const int nb = nblk(ntiles, SH_BLOCK / SH_WAVE);
  if (nb > 0) {
    if (prec == 0) hipLaunchKernelGGL(k_absmax<double>, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, part);
    else hipLaunchKernelGGL(k_absmax<float>, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, part);
  }
  hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(256), 0, st, part, ntiles, out);
}

void sh_launch_poison_ghosts(int prec, const BoxDev* boxes, int nboxes, int nplanes, int ng, int role, int ncomp,
                             hipStream_t st) {
  if (nboxes == 0 || nplanes == 0) return;
  const unsigned nb = (unsigned)nboxes * (unsigned)nplanes;
  if (prec == 0)
    hipLaunchKernelGGL(k_poison_ghosts<double>, dim3(nb), dim3(SH_BLOCK), 0, st, boxes, nplanes, ng, role, ncomp);
  else
    hipLaunchKernelGGL(k_poison_ghosts<float>, dim3(nb), dim3(SH_BLOCK), 0, st, boxes, nplanes, ng, role, ncomp);
}

void sh_launch_counter_zero(LevelScal* ls, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_counter_zero, dim3(nblk(n, 64)), dim3(64), 0, st, ls, n);
}

