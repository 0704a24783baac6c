// Internal device/host structures of libshamr (not part of the public C-ABI).
//
// Storage of one box (all levels, all buffers): structure-of-arrays
//   element(c, i, j, k) = off + c*cs + ((k+ng)*py + (j+ng))*px + XOFF + i
// for component c in {psi1, psi2, Pi1, Pi2}, box-local cell (i, j, k) with
// -ng <= i < nx + ng etc. (a ghost shell ng cells deep: 1 on refined levels, 4 on
// level 0 so that four RK stages can be fused).  XOFF puts i = 0 on a 64-byte boundary
// and px is a multiple of XOFF, so every x-row of valid cells starts 64-byte aligned.
// A level owns three state slots of this layout in the storage precision T plus one
// float64 accumulator slot with the same element offsets.
#pragma once
#include <stdint.h>

#define SH_WAVE 64
#define SH_BLOCK 256

// Per-level scalars on the device.  k is the number of steps the level has taken; the
// level time is eta0 + k*dt (one multiply and one add, so aligned levels hold
// bit-identical times).  nst is the number of stages per step of the integrator (4:
// classic RK4, 3: SSPRK3).  Every kernel resolves buffer roles from k and nst, so a
// launch sequence can be replayed without host updates.  ko is the coefficient of the
// Kreiss-Oliger sum on this level (-eps/(16 dx) or eps/(64 dx); 0 without dissipation).
struct LevelScal {
  double eta0, dt, alpha, lam, inv_dx2, dx, ko;
  int beta, nst;
  long long k;
};

// Buffer roles.
// RK4, with p = k & 1: U_n = slot[2p], A = slot[1], B = slot[2 - 2p].  The stages read
// (U_n, A, B, A) and write (A, B, A, B); after stage 4 and the counter increment, the
// old U_n (OLD) is slot B of the new parity until the next stage 2.
// SSPRK3, with q = k mod 3: U_n = slot[q], A = slot[q+1], B = slot[q+2] (mod 3).  The
// stages read (U_n, A, B) and write (A, B, A): the new state lands in slot[q+1], which
// is U_n of step k+1, and the old U_n is then slot B = slot[(k+1)+2] until the next
// stage 2 overwrites it.
enum { ROLE_UN = 0, ROLE_A = 1, ROLE_B = 2, ROLE_OLD = 3 };

// k mod 3 for k >= 0 from 32-bit halves (2^32 = 1 mod 3): a 64-bit division would be
// expanded into a long vector sequence in every kernel that resolves a role.
__host__ __device__ inline int mod3(long long k) {
  const unsigned long long u = (unsigned long long)k;
  return (int)(((unsigned)u % 3u + (unsigned)(u >> 32) % 3u) % 3u);
}

// RKN5 (nst = 5 here: four stages over three slots): U_n = slot[q] with q = 2k mod 3, A =
// slot[q+1], B = slot[q+2]; the stages read (U_n, A, B, A) and write (A, B, A, B), so
// U_{n+1} lands in slot[q+2] = slot[2(k+1) mod 3].
__host__ __device__ inline int role_slot(int role, long long k, int nst) {
  if (nst == 5) {
    const int q = mod3(2 * k);
    if (role == ROLE_UN) return q;
    if (role == ROLE_B) return q == 0 ? 2 : q - 1;
    return q == 2 ? 0 : q + 1;  // ROLE_A and ROLE_OLD
  }
  if (nst == 3) {
    const int q = mod3(k);
    if (role == ROLE_UN) return q;
    if (role == ROLE_A) return q == 2 ? 0 : q + 1;
    return q == 0 ? 2 : q - 1;  // ROLE_B and ROLE_OLD
  }
  const int p = (int)(k & 1);
  switch (role) {
    case ROLE_UN: return 2 * p;
    case ROLE_A: return 1;
    case ROLE_B: return 2 - 2 * p;
    default: return 2 - 2 * p;  // ROLE_OLD (valid once k has been incremented)
  }
}

__host__ __device__ inline int role_slot(int role, const LevelScal& L) { return role_slot(role, L.k, L.nst); }

// Stage ids of the kernels: 0..3 the four RK4 stages, 4..6 the three SSPRK3 stages.
// Fraction c_s of the step at which each evaluates the right-hand side:
// RK4 (0, 1/2, 1/2, 1), SSPRK3 (0, 1, 1/2).
// c_s of stage id s: RK4 ids 0..3 (0, 1/2, 1/2, 1), SSPRK3 ids 4..6 (0, 1, 1/2), RKN4 ids
// 7..9 (0, 1/2, 1), RKN5 ids 10..13 (0, 1/5, 2/3, 1).
__host__ __device__ inline double stage_frac(int s) {
  if (s >= 10) return s == 10 ? 0.0 : (s == 11 ? 0.2 : (s == 12 ? 2.0 / 3.0 : 1.0));
  return (s == 0 || s == 4 || s == 7) ? 0.0 : ((s == 3 || s == 5 || s == 9) ? 1.0 : 0.5);
}

struct BoxDev {
  void* slot[3];      // base of this box's storage block in each state slot (type T)
  double* acc;        // base of this box's block in the accumulator slot
  LevelScal* ls;      // scalars of the box's level
  long long cs;       // component stride (elements)
  int nx, ny, nz;     // valid cells
  int px, py;         // x pitch (elements), y pitch (ny + 2)
  int lo[3];          // global index of cell (0,0,0) on the box's level
  int mask_off;       // offset of the box's valid cells in per-level byte masks
  int ng;             // ghost layers stored around the box
  int xoff;           // elements before x = 0 in a row
};

// Wave tile: one wavefront covers a TX x (64/TX) footprint of a box and marches in z.
struct Tile {
  int box;
  int xy;   // x0 | y0 << 16
  int zz;   // z0 | zc << 16
  int txs;  // log2(TX)
};

// Same-level ghost copy (psi components): dst region (box-local, inside the ghost
// shell) <- src region (box-local, valid cells of src box).
struct CopySeg {
  int dbox, sbox;
  int dlo[3], slo[3], n[3];
  int pad;
};

// Coarse->fine interpolation: fine cells of region flo..flo+n-1 (fine box-local) whose
// global index is fg = flo + fglo_minus_flo; parent in coarse box-local coordinates
// is floor(fg/2) + cshift.
struct InterpSeg {
  int fbox, cbox;
  int flo[3], n[3];
  int fg0[3];      // global fine index of flo
  int cshift[3];   // coarse local = floor(fg/2) + cshift
};

// Coarse-to-fine interpolation works on tiles of parent cells of a segment (one workgroup
// each, the time-interpolated coarse support in LDS); its block plan lists tile t of a
// segment as SegBlock{seg, t * SH_BLOCK}.  Tile extents: the segment's parent extents
// capped at 16, the largest halved until at most SH_BLOCK parents remain (thin ghost
// shells get wide, flat tiles).  The support (extents + 4 for the quartic reach of two
// cells) then holds at most QT_LDS values.
#define QT_LDS 2000
__host__ __device__ inline void qtile_dims(const int np[3], int t[3]) {
  for (int d = 0; d < 3; ++d) t[d] = np[d] < 16 ? np[d] : 16;
  while (t[0] * t[1] * t[2] > SH_BLOCK) {
    int m = 0;
    if (t[1] > t[m]) m = 1;
    if (t[2] > t[m]) m = 2;
    t[m] = (t[m] + 1) / 2;
  }
}

// Average down: coarse cells clo..clo+n-1 (coarse box-local) of box cbox from fine box
// fbox whose child (0,0,0) of coarse cell clo sits at fine-local f0.
struct AvgSeg {
  int cbox, fbox;
  int clo[3], n[3], f0[3];
  int pad;
};

// Flat work decomposition of a segment list: block b covers cells
// [start, start + SH_BLOCK) of segment seg.
struct SegBlock {
  int seg, start;
};

// Per-wave-tile partial reduction of the energy and the non-finite count.
struct EnergyPartial {
  double kin, grad, pot;
  long long nonfinite;
};

// Truncation error estimates kept per cell: nc = 1 (the maximum over the components) or
// 4 (one per component, component c at tee + c * cs, cs = the level's valid cells).
// Tagging by estimate: nc = 1 tags where tee > crit[0]; nc = 4 where
// scale[c] * tee_c > crit[c] for some component (the modifier f_c(D) = scale_c D).
struct TeeSpec {
  double crit[4];
  double scale[4];
  int nc;
  long long cs;
};

