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

#pragma clang fp contract(off)

// ---------------------------------------------------------------------------------
// A3: fused RK4 stage.
//   lap   = ((((u[x-1]+u[x+1]) + (u[y-1]+u[y+1])) + (u[z-1]+u[z+1])) - 6u) * inv_dx2
//   k_psi = Pi,  k_Pi = (lap - c_fric Pi) - c_pot (r2 - 1) psi
//   stage 1: acc = U_n + h/6 k;   A = U_n + h/2 k
//   stage 2: acc = acc + h/3 k;   B = U_n + h/2 k
//   stage 3: acc = acc + h/3 k;   A = U_n + h k
//   stage 4: B = acc + h/6 k      (the new U_n)
// SSPRK3 (stage ids 4..6; appendix E's three-stage strong-stability-preserving method
// in Shu-Osher form):
//   stage 1: A = U_n + h k
//   stage 2: B = 3/4 U_n + 1/4 (A + h k)
//   stage 3: A = 1/3 U_n + 2/3 (B + h k)   (the new U_n)
// The right-hand side is evaluated in T; updates in float64, rounded to T on store.
// NT = 1 marks the streams read or written once (Pi, U_n, acc, the stage output) as
// nontemporal so they do not push the psi planes, which neighbours re-read, out of L2.
// ---------------------------------------------------------------------------------
struct StagePtrs {
  const void* X;
  const void* Un;
  void* Y;
  double* acc;
};

template <typename T, int S>
__device__ __forceinline__ StagePtrs stage_ptrs(const BoxDev& B, const LevelScal& L) {
  constexpr int in_role = (S == 0 || S == 4) ? ROLE_UN : ((S == 2 || S == 6) ? ROLE_B : ROLE_A);
  constexpr int out_role = (S == 1 || S == 3 || S == 5) ? ROLE_B : ROLE_A;
  StagePtrs p;
  p.X = slot_base(B, role_slot(in_role, L));
  p.Un = slot_base(B, role_slot(ROLE_UN, L));
  p.Y = slot_base(B, role_slot(out_role, L));
  p.acc = B.acc;
  return p;
}

// Per-cell right-hand side and stage update.  p0/p1 = psi at the cell, lap0/lap1 their
// Laplacians, q0/q1 = Pi at the cell (all in T); e = element index of the cell.
template <typename T, int S, bool NT>
__device__ __forceinline__ void stage_cell(const StageScal& sc, const T* __restrict__ Un, T* __restrict__ Y,
                                           double* __restrict__ acc, long long cs, long long e, T p0, T p1,
                                           T q0, T q1, T lap0, T lap1, const double* un4, const double* acc4) {
  const T cf = (T)sc.cf, cp = (T)sc.cp;
  const T r2 = p0 * p0 + p1 * p1;
  const T pot = cp * (r2 - (T)1.0);
  const T kq0 = (lap0 - cf * q0) - pot * p0;
  const T kq1 = (lap1 - cf * q1) - pot * p1;
  const double k4[4] = {(double)q0, (double)q1, (double)kq0, (double)kq1};
  const T xv[4] = {p0, p1, q0, q1};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const long long ec = c * cs + e;
    if constexpr (S == 0) {
      const double u = (double)xv[c];
      st<NT>(acc + ec, u + sc.h6 * k4[c]);
      st<NT>(Y + ec, (T)(u + sc.h2 * k4[c]));
    } else if constexpr (S == 1 || S == 2) {
      st<NT>(acc + ec, acc4[c] + sc.h3 * k4[c]);
      st<NT>(Y + ec, (T)(un4[c] + (S == 1 ? sc.h2 : sc.h1) * k4[c]));
    } else if constexpr (S == 3) {
      st<NT>(Y + ec, (T)(acc4[c] + sc.h6 * k4[c]));
    } else if constexpr (S == 4) {
      st<NT>(Y + ec, (T)((double)xv[c] + sc.h1 * k4[c]));
    } else if constexpr (S == 5) {
      st<NT>(Y + ec, (T)(0.75 * un4[c] + 0.25 * ((double)xv[c] + sc.h1 * k4[c])));
    } else {
      st<NT>(Y + ec, (T)((1.0 / 3.0) * un4[c] + (2.0 / 3.0) * ((double)xv[c] + sc.h1 * k4[c])));
    }
  }
}

// Loads of the once-read streams of a cell: U_n (RK4 stages 2, 3; SSPRK3 stages 2, 3)
// and acc (RK4 stages 2-4).
template <typename T, int S, bool NT>
__device__ __forceinline__ void stage_loads(const T* __restrict__ Un, const double* __restrict__ acc, long long cs,
                                            long long e, double* un4, double* acc4) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if constexpr (S == 1 || S == 2 || S == 5 || S == 6) un4[c] = (double)ld<NT>(Un + c * cs + e);
    if constexpr (S >= 1 && S <= 3) acc4[c] = ld<NT>(acc + c * cs + e);
  }
}

// Wave-row kernel: one wavefront per tile (a TX x 64/TX footprint of a box, marching
// in z); psi(z-1), psi(z), psi(z+1) of both components stay in registers, x and y
// neighbours are read through the caches.  Used for boxes narrower than 64 cells.
template <typename T, int S, bool NT>
__global__ __launch_bounds__(SH_BLOCK) void k_stage(const Tile* __restrict__ tiles, int ntiles,
                                                    const BoxDev* __restrict__ boxes) {
  const int lane = threadIdx.x & (SH_WAVE - 1);
  const int t = xcd_remap(blockIdx.x, gridDim.x) * (SH_BLOCK / SH_WAVE) + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const Tile tl = tiles[t];
  if (tl.box < 0) return;
  const BoxDev B = boxes[tl.box];
  const LevelScal L = *B.ls;
  const StageScal sc = stage_scalars(L, S);
  const StagePtrs P = stage_ptrs<T, S>(B, L);
  const T* __restrict__ X = (const T*)P.X;
  const T* __restrict__ Un = (const T*)P.Un;
  T* __restrict__ Y = (T*)P.Y;

  const int tx = lane & ((1 << tl.txs) - 1);
  const int ty = lane >> tl.txs;
  const int x0 = tl.xy & 0xffff, y0 = tl.xy >> 16;
  const int z0 = tl.zz & 0xffff, zc = tl.zz >> 16;
  int x = x0 + tx, y = y0 + ty;
  const bool active = (x < B.nx) && (y < B.ny);
  x = min(x, B.nx - 1);
  y = min(y, B.ny - 1);
  const long long px = B.px;
  const long long plane = px * B.py;
  const long long cs = B.cs;
  const int zend = min(z0 + zc, B.nz);
  const T idx2 = (T)sc.inv_dx2;

  long long e = elem<T>(B, x, y, z0);
  T pm0 = X[e - plane], p00 = X[e];
  T pm1 = X[cs + e - plane], p01 = X[cs + e];
  for (int z = z0; z < zend; ++z, e += plane) {
    const T pp0 = X[e + plane];
    const T pp1 = X[cs + e + plane];
    const T xm0 = X[e - 1], xp0 = X[e + 1], ym0 = X[e - px], yp0 = X[e + px];
    const T xm1 = X[cs + e - 1], xp1 = X[cs + e + 1], ym1 = X[cs + e - px], yp1 = X[cs + e + px];
    const T q0 = ld<NT>(X + 2 * cs + e), q1 = ld<NT>(X + 3 * cs + e);
    double un4[4], acc4[4];
    stage_loads<T, S, NT>(Un, P.acc, cs, e, un4, acc4);
    const T lap0 = ((((xm0 + xp0) + (ym0 + yp0)) + (pm0 + pp0)) - (T)6.0 * p00) * idx2;
    const T lap1 = ((((xm1 + xp1) + (ym1 + yp1)) + (pm1 + pp1)) - (T)6.0 * p01) * idx2;
    if (active) stage_cell<T, S, NT>(sc, Un, Y, P.acc, cs, e, p00, p01, q0, q1, lap0, lap1, un4, acc4);
    pm0 = p00; p00 = pp0;
    pm1 = p01; p01 = pp1;
  }
}

// Block-row kernel for boxes at least 64 cells wide: a block of R wavefronts covers a
// 64 x R footprint (wave w owns row y0 + w) and marches in z in lock step.  Each wave
// keeps psi(z-1..z+1) of its own row in registers and publishes psi(z) of the row to LDS,
// where the rows above and below (and the two x-halo columns, loaded by the edge lanes;
// the halo rows y0-1 and y0+R, loaded by the first and last wave) are read back.  psi is
// therefore fetched about (R+2)/R times per plane instead of five times through the caches.
template <typename T, int S, bool NT, int R>
__global__ __launch_bounds__(SH_WAVE * R) void k_stage_lds(const Tile* __restrict__ tiles, int ntiles,
                                                           const BoxDev* __restrict__ boxes) {
  __shared__ T sm[2][2][R + 2][SH_WAVE + 2];
  const int lane = threadIdx.x & (SH_WAVE - 1);
  const int w = threadIdx.x >> 6;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  if (t >= ntiles) return;  // uniform over the block
  const Tile tl = tiles[t];
  if (tl.box < 0) return;
  const BoxDev B = boxes[tl.box];
  const LevelScal L = *B.ls;
  const StageScal sc = stage_scalars(L, S);
  const StagePtrs P = stage_ptrs<T, S>(B, L);
  const T* __restrict__ X = (const T*)P.X;
  const T* __restrict__ Un = (const T*)P.Un;
  T* __restrict__ Y = (T*)P.Y;

  const int x0 = tl.xy & 0xffff, y0 = tl.xy >> 16;
  const int z0 = tl.zz & 0xffff, zc = tl.zz >> 16;
  const int x = x0 + lane, y = y0 + w;
  const bool active = (x < B.nx) && (y < B.ny);
  // rows and columns past the box edge load the ghost row/column instead (valid memory)
  const int xl = min(x, B.nx), yl = min(y, B.ny);
  const long long px = B.px;
  const long long plane = px * B.py;
  const long long cs = B.cs;
  const int zend = min(z0 + zc, B.nz);
  const T idx2 = (T)sc.inv_dx2;

  long long e = elem<T>(B, xl, yl, z0);
  // halo row below (wave 0) / above (wave R-1), x-halo columns (lanes 0 / 63)
  const long long eh = (w == 0) ? elem<T>(B, xl, y0 - 1, z0) : elem<T>(B, xl, min(y0 + R, B.ny), z0);
  const bool has_h = (w == 0) || (w == R - 1);
  const long long ex = (lane == 0) ? elem<T>(B, x0 - 1, yl, z0) : elem<T>(B, min(x0 + SH_WAVE, B.nx), yl, z0);
  const bool has_x = (lane == 0) || (lane == SH_WAVE - 1);
  const int hrow = (w == 0) ? 0 : R + 1;
  const int xcol = (lane == 0) ? 0 : SH_WAVE + 1;

  T pm[2], p0[2], pp[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    pm[c] = X[c * cs + e - plane];
    p0[c] = X[c * cs + e];
  }
  int buf = 0;
  for (int z = z0; z < zend; ++z, e += plane, buf ^= 1) {
    const long long zo = (long long)(z - z0) * plane;
    T hv[2] = {(T)0, (T)0}, xv[2] = {(T)0, (T)0};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      pp[c] = X[c * cs + e + plane];
      if (has_h) hv[c] = X[c * cs + eh + zo];
      if (has_x) xv[c] = X[c * cs + ex + zo];
    }
    const T q0 = ld<NT>(X + 2 * cs + e), q1 = ld<NT>(X + 3 * cs + e);
    double un4[4], acc4[4];
    stage_loads<T, S, NT>(Un, P.acc, cs, e, un4, acc4);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      sm[buf][c][w + 1][lane + 1] = p0[c];
      if (has_h) sm[buf][c][hrow][lane + 1] = hv[c];
      if (has_x) sm[buf][c][w + 1][xcol] = xv[c];
    }
    lds_barrier();
    T lap[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const T xm = sm[buf][c][w + 1][lane], xp = sm[buf][c][w + 1][lane + 2];
      const T ym = sm[buf][c][w][lane + 1], yp = sm[buf][c][w + 2][lane + 1];
      lap[c] = ((((xm + xp) + (ym + yp)) + (pm[c] + pp[c])) - (T)6.0 * p0[c]) * idx2;
    }
    if (active) stage_cell<T, S, NT>(sc, Un, Y, P.acc, cs, e, p0[0], p0[1], q0, q1, lap[0], lap[1], un4, acc4);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      pm[c] = p0[c];
      p0[c] = pp[c];
    }
  }
}

// Right-hand side only (diagnostic): out[box][c][z][y][x] = f(U_n) at stage-1 scalars.
template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_rhs(const Tile* __restrict__ tiles, int ntiles,
                                                  const BoxDev* __restrict__ boxes,
                                                  const long long* __restrict__ out_off,
                                                  double* __restrict__ out) {
  const int lane = threadIdx.x & (SH_WAVE - 1);
  const int t = blockIdx.x * (SH_BLOCK / SH_WAVE) + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const Tile tl = tiles[t];
  if (tl.box < 0) return;
  const BoxDev B = boxes[tl.box];
  const LevelScal L = *B.ls;
  const StageScal sc = stage_scalars(L, 0);
  const T* __restrict__ X = (const T*)slot_base(B, role_slot(ROLE_UN, L));
  const int tx = lane & ((1 << tl.txs) - 1), ty = lane >> tl.txs;
  const int x = (tl.xy & 0xffff) + tx, y = (tl.xy >> 16) + ty;
  if (x >= B.nx || y >= B.ny) return;
  const int z0 = tl.zz & 0xffff, zend = min(z0 + (tl.zz >> 16), B.nz);
  const long long px = B.px, plane = px * B.py, cs = B.cs;
  const long long nv = (long long)B.nx * B.ny * B.nz;
  const T cf = (T)sc.cf, cp = (T)sc.cp, idx2 = (T)sc.inv_dx2;
  for (int z = z0; z < zend; ++z) {
    const long long e = elem<T>(B, x, y, z);
    T lap[2];
    for (int c = 0; c < 2; ++c) {
      const T* u = X + c * cs;
      lap[c] = ((((u[e - 1] + u[e + 1]) + (u[e - px] + u[e + px])) + (u[e - plane] + u[e + plane])) -
                (T)6.0 * u[e]) * idx2;
    }
    const T p0 = X[e], p1 = X[cs + e], q0 = X[2 * cs + e], q1 = X[3 * cs + e];
    const T r2 = p0 * p0 + p1 * p1;
    const T pot = cp * (r2 - (T)1.0);
    const long long o = out_off[tl.box] + ((long long)z * B.ny + y) * B.nx + x;
    out[o] = (double)q0;
    out[o + nv] = (double)q1;
    out[o + 2 * nv] = (double)((lap[0] - cf * q0) - pot * p0);
    out[o + 3 * nv] = (double)((lap[1] - cf * q1) - pot * p1);
  }
}

__global__ void k_counter_inc_list(LevelScal* const* ls, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ls[i]->k += 1;
}

__global__ void k_counter_inc(LevelScal* ls, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ls[i].k += 1;
}

// ---------------------------------------------------------------------------------
// A1: same-level ghost copy (periodic images included) of the first ncomp components:
// the psi pair on the stepping path, all four before a regrid interpolates from them.
// ---------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_ghost_copy(const CopySeg* __restrict__ segs,
                                                         const SegBlock* __restrict__ blocks,
                                                         const BoxDev* __restrict__ boxes, int role, int ncomp) {
  const SegBlock sb = blocks[blockIdx.x];
  const CopySeg s = segs[sb.seg];
  const int c = sb.start + threadIdx.x;
  if (c >= s.n[0] * s.n[1] * s.n[2]) return;
  const int i = c % s.n[0];
  const int r = c / s.n[0];
  const int j = r % s.n[1];
  const int k = r / s.n[1];
  const BoxDev& D = boxes[s.dbox];
  const BoxDev& Sb = boxes[s.sbox];
  const int sl = role_slot(role, *D.ls);
  T* dst = (T*)D.slot[sl];
  const T* src = (const T*)Sb.slot[sl];
  const long long ed = elem<T>(D, s.dlo[0] + i, s.dlo[1] + j, s.dlo[2] + k);
  const long long es = elem<T>(Sb, s.slo[0] + i, s.slo[1] + j, s.slo[2] + k);
  for (int comp = 0; comp < ncomp; ++comp) dst[comp * D.cs + ed] = src[comp * Sb.cs + es];
}

// ---------------------------------------------------------------------------------
// A2: coarse->fine ghost interpolation of the psi components.  Time first:
//   C(alpha) = (1 - alpha) C_old + alpha C_new  (alpha = 0, 1: the stored state itself)
// then linear conservative space interpolation with central slopes:
//   f = ((C_I + t_x) + t_y) + t_z,  t_d = (C_{I+e_d} - C_{I-e_d}) * (+-1/8)
// Arithmetic in float64, rounded to T on store.
// ---------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double tinterp(const T* Cold, const T* Cnew, long long e, int anum, double a) {
  if (anum == 4) return (double)Cnew[e];
  if (anum == 0) return (double)Cold[e];
  return (1.0 - a) * (double)Cold[e] + a * (double)Cnew[e];
}

template <typename T>
__device__ __forceinline__ double interp_one(const BoxDev& C, const T* Cold, const T* Cnew, int ci, int cj,
                                             int ck, int fx, int fy, int fz, int anum) {
  const double a = 0.25 * (double)anum;
  const long long px = C.px, plane = px * C.py;
  const long long e = elem<T>(C, ci, cj, ck);
  const double c0 = tinterp(Cold, Cnew, e, anum, a);
  const double sx = (fx & 1) ? 0.125 : -0.125;
  const double sy = (fy & 1) ? 0.125 : -0.125;
  const double sz = (fz & 1) ? 0.125 : -0.125;
  const double tx = (tinterp(Cold, Cnew, e + 1, anum, a) - tinterp(Cold, Cnew, e - 1, anum, a)) * sx;
  const double ty = (tinterp(Cold, Cnew, e + px, anum, a) - tinterp(Cold, Cnew, e - px, anum, a)) * sy;
  const double tz = (tinterp(Cold, Cnew, e + plane, anum, a) - tinterp(Cold, Cnew, e - plane, anum, a)) * sz;
  return ((c0 + tx) + ty) + tz;
}

template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_ghost_interp(const InterpSeg* __restrict__ segs,
                                                           const SegBlock* __restrict__ blocks,
                                                           const BoxDev* __restrict__ fboxes,
                                                           const BoxDev* __restrict__ cboxes, int role,
                                                           int anum, int ncomp) {
  const SegBlock sb = blocks[blockIdx.x];
  const InterpSeg s = segs[sb.seg];
  const int c = sb.start + threadIdx.x;
  if (c >= s.n[0] * s.n[1] * s.n[2]) return;
  const int i = c % s.n[0];
  const int r = c / s.n[0];
  const int j = r % s.n[1];
  const int k = r / s.n[1];
  const BoxDev& F = fboxes[s.fbox];
  const BoxDev& C = cboxes[s.cbox];
  const LevelScal& LC = *C.ls;
  const T* Cnew = (const T*)C.slot[role_slot(ROLE_UN, LC)];
  const T* Cold = (const T*)C.slot[role_slot(ROLE_OLD, LC)];
  T* dst = (T*)F.slot[role_slot(role, *F.ls)];
  const int fx = s.fg0[0] + i, fy = s.fg0[1] + j, fz = s.fg0[2] + k;
  const int ci = (fx >> 1) + s.cshift[0], cj = (fy >> 1) + s.cshift[1], ck = (fz >> 1) + s.cshift[2];
  const long long ed = elem<T>(F, s.flo[0] + i, s.flo[1] + j, s.flo[2] + k);
  for (int comp = 0; comp < ncomp; ++comp) {
    const double v = interp_one<T>(C, Cold + comp * C.cs, Cnew + comp * C.cs, ci, cj, ck, fx, fy, fz, anum);
    dst[comp * F.cs + ed] = (T)v;
  }
}

// ---------------------------------------------------------------------------------
// A5: average down, all 4 components, fine U_n -> coarse U_n:
//   c = ((((f000+f100)+(f010+f110))+((f001+f101)+(f011+f111))) * 0.125)
// With tee: first the truncation error estimate, max over the components of
// |C - avg| (float64; the first component's value unless a later one compares greater),
// stored on the 8 children in the fine level's per-cell array.  write_coarse = 0 keeps
// the coarse state (the shadow-level comparison).
// ---------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_avgdown(const AvgSeg* __restrict__ segs,
                                                      const SegBlock* __restrict__ blocks,
                                                      const BoxDev* __restrict__ cboxes,
                                                      const BoxDev* __restrict__ fboxes, double* __restrict__ tee,
                                                      int write_coarse) {
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
  T* dst = (T*)slot_base(C, role_slot(ROLE_UN, *C.ls));
  const T* src = (const T*)slot_base(F, role_slot(ROLE_UN, *F.ls));
  const long long ec = elem<T>(C, s.clo[0] + i, s.clo[1] + j, s.clo[2] + k);
  const long long ef = elem<T>(F, s.f0[0] + 2 * i, s.f0[1] + 2 * j, s.f0[2] + 2 * k);
  const long long px = F.px, plane = px * F.py;
  double t = 0.0;
  for (int comp = 0; comp < 4; ++comp) {
    const T* f = src + comp * F.cs + ef;
    const double f000 = f[0], f100 = f[1], f010 = f[px], f110 = f[px + 1];
    const double f001 = f[plane], f101 = f[plane + 1], f011 = f[plane + px], f111 = f[plane + px + 1];
    const double avg = ((((f000 + f100) + (f010 + f110)) + ((f001 + f101) + (f011 + f111))) * 0.125);
    if (tee) {
      const double d = fabs((double)dst[comp * C.cs + ec] - avg);
      t = (comp == 0 || d > t) ? d : t;
    }
    if (write_coarse) dst[comp * C.cs + ec] = (T)avg;
  }
  if (tee) {
    const int x0 = s.f0[0] + 2 * i, y0 = s.f0[1] + 2 * j, z0 = s.f0[2] + 2 * k;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy) {
        const long long row = F.mask_off + ((long long)(z0 + dz) * F.ny + (y0 + dy)) * F.nx + x0;
        tee[row] = t;
        tee[row + 1] = t;
      }
  }
}

// Regrid: copy the 4 components of valid cells from the old layout of a level.
template <typename T>
__global__ __launch_bounds__(SH_BLOCK) void k_regrid_copy(const CopySeg* __restrict__ segs,
                                                          const SegBlock* __restrict__ blocks,
                                                          const BoxDev* __restrict__ dboxes,
                                                          const BoxDev* __restrict__ sboxes,
                                                          const double* __restrict__ tee_src,
                                                          double* __restrict__ tee_dst) {
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
  if (tee_src)
    tee_dst[D.mask_off + ((long long)(s.dlo[2] + k) * D.ny + (s.dlo[1] + j)) * D.nx + (s.dlo[0] + i)] =
        tee_src[Sb.mask_off + ((long long)(s.slo[2] + k) * Sb.ny + (s.slo[1] + j)) * Sb.nx + (s.slo[0] + i)];
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
                                                  double te_crit, int mode) {
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
    bool tag = (mode & 2) && tee[cell] > te_crit;
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

template <typename T, int S, bool NT>
static void stage_launch3(int kind, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  if (ntiles == 0) return;
  if (kind == 0) {
    hipLaunchKernelGGL((k_stage<T, S, NT>), dim3(nblk(ntiles, SH_BLOCK / SH_WAVE)), dim3(SH_BLOCK), 0, st, tiles,
                       ntiles, boxes);
  } else if (kind == 4) {
    hipLaunchKernelGGL((k_stage_lds<T, S, NT, 4>), dim3(ntiles), dim3(SH_WAVE * 4), 0, st, tiles, ntiles, boxes);
  } else {
    hipLaunchKernelGGL((k_stage_lds<T, S, NT, 8>), dim3(ntiles), dim3(SH_WAVE * 8), 0, st, tiles, ntiles, boxes);
  }
}

template <typename T, bool NT>
static void stage_launch2(int s, int kind, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  switch (s) {
    case 0: stage_launch3<T, 0, NT>(kind, tiles, ntiles, boxes, st); break;
    case 1: stage_launch3<T, 1, NT>(kind, tiles, ntiles, boxes, st); break;
    case 2: stage_launch3<T, 2, NT>(kind, tiles, ntiles, boxes, st); break;
    case 3: stage_launch3<T, 3, NT>(kind, tiles, ntiles, boxes, st); break;
    case 4: stage_launch3<T, 4, NT>(kind, tiles, ntiles, boxes, st); break;
    case 5: stage_launch3<T, 5, NT>(kind, tiles, ntiles, boxes, st); break;
    default: stage_launch3<T, 6, NT>(kind, tiles, ntiles, boxes, st); break;
  }
}

// kind: 0 = wave-row tiles (k_stage), 4 or 8 = block-row tiles of that many rows
void sh_launch_stage(int prec, int s, int kind, bool nt, const Tile* tiles, int ntiles, const BoxDev* boxes,
                     hipStream_t st) {
  if (prec == 0) {
    if (nt) stage_launch2<double, true>(s, kind, tiles, ntiles, boxes, st);
    else stage_launch2<double, false>(s, kind, tiles, ntiles, boxes, st);
  } else {
    if (nt) stage_launch2<float, true>(s, kind, tiles, ntiles, boxes, st);
    else stage_launch2<float, false>(s, kind, tiles, ntiles, boxes, st);
  }
}

void sh_launch_rhs(int prec, const Tile* tiles, int ntiles, const BoxDev* boxes, const long long* out_off,
                   double* out, hipStream_t st) {
  const int nb = nblk(ntiles, SH_BLOCK / SH_WAVE);
  if (nb == 0) return;
  if (prec == 0) hipLaunchKernelGGL(k_rhs<double>, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, out_off, out);
  else hipLaunchKernelGGL(k_rhs<float>, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, out_off, out);
}

void sh_launch_counter_inc_list(LevelScal* const* ls, int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_counter_inc_list, dim3(nblk(n, 64)), dim3(64), 0, st, ls, n);
}

void sh_launch_counter_inc(LevelScal* ls, int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_counter_inc, dim3(nblk(n, 64)), dim3(64), 0, st, ls, n);
}

void sh_launch_ghost_copy(int prec, const CopySeg* segs, const SegBlock* blocks, int nblocks, const BoxDev* boxes,
                          int role, int ncomp, hipStream_t st) {
  if (nblocks == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL(k_ghost_copy<double>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, boxes, role, ncomp);
  else
    hipLaunchKernelGGL(k_ghost_copy<float>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, boxes, role, ncomp);
}

void sh_launch_ghost_interp(int prec, const InterpSeg* segs, const SegBlock* blocks, int nblocks,
                            const BoxDev* fboxes, const BoxDev* cboxes, int role, int anum, int ncomp,
                            hipStream_t st) {
  if (nblocks == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL(k_ghost_interp<double>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, fboxes, cboxes, role,
                       anum, ncomp);
  else
    hipLaunchKernelGGL(k_ghost_interp<float>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, fboxes, cboxes, role,
                       anum, ncomp);
}

void sh_launch_avgdown(int prec, const AvgSeg* segs, const SegBlock* blocks, int nblocks, const BoxDev* cboxes,
                       const BoxDev* fboxes, double* tee, int write_coarse, hipStream_t st) {
  if (nblocks == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL(k_avgdown<double>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, cboxes, fboxes, tee,
                       write_coarse);
  else
    hipLaunchKernelGGL(k_avgdown<float>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, cboxes, fboxes, tee,
                       write_coarse);
}

void sh_launch_regrid_copy(int prec, const CopySeg* segs, const SegBlock* blocks, int nblocks, const BoxDev* dboxes,
                           const BoxDev* sboxes, const double* tee_src, double* tee_dst, hipStream_t st) {
  if (nblocks == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL(k_regrid_copy<double>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, dboxes, sboxes,
                       tee_src, tee_dst);
  else
    hipLaunchKernelGGL(k_regrid_copy<float>, dim3(nblocks), dim3(SH_BLOCK), 0, st, segs, blocks, dboxes, sboxes,
                       tee_src, tee_dst);
}

void sh_launch_tag(int prec, const Tile* tiles, int ntiles, const BoxDev* boxes, uint8_t* mask, int* tile_count,
                   const double* tee, double te_crit, int mode, hipStream_t st) {
  const int nb = nblk(ntiles, SH_BLOCK / SH_WAVE);
  if (nb == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL(k_tag<double>, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, mask, tile_count, tee,
                       te_crit, mode);
  else
    hipLaunchKernelGGL(k_tag<float>, dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, mask, tile_count, tee,
                       te_crit, mode);
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
