// Per-stage kernels of the level step (internal), templated on the stencil radius H:
// the Laplacian of appendix A at order H = 1, 2, 3 (7-, 13-, 19-point).  Included by
// kernels.hip (H = 1) and kernels_hilap.hip (H = 2, 3), which instantiate them.
//
// A3: stage kernel.  With S_r the sum of the six cells at distance r,
//   S_r   = ((u[x-r]+u[x+r]) + (u[y-r]+u[y+r])) + (u[z-r]+u[z+r])
//   lap   = (S_1 - 6u) * inv_dx2                                           H = 1
//         = ((4/3 S_1 + (-1/12) S_2) + (-15/2) u) * inv_dx2                  H = 2
//         = (((3/2 S_1 + (-3/20) S_2) + 1/90 S_3) + (-49/6) u) * inv_dx2     H = 3
//   (coefficients rounded once to T)
//   k_psi = Pi,  k_Pi = (lap - c_fric Pi) - c_pot (r2 - 1) psi
// RK4 (stage ids 0..3):
//   stage 1: acc = U_n + h/6 k;   A = U_n + h/2 k
//   stage 2: acc = acc + h/3 k;   B = U_n + h/2 k
//   stage 3: acc = acc + h/3 k;   A = U_n + h k
//   stage 4: B = acc + h/6 k      (the new U_n)
// SSPRK3 (stage ids 4..6; appendix E's three-stage strong-stability-preserving method
// in Shu-Osher form):
//   stage 1: A = U_n + h k
//   stage 2: B = 3/4 U_n + 1/4 (A + h k)
//   stage 3: A = 1/3 U_n + 2/3 (B + h k)   (the new U_n)
// RKN4 (stage ids 7..9; appendix E's integrator type 21, read as Nystrom's classical
// three-stage fourth-order method for psi'' = a(psi), which needs alpha = 0 and no
// dissipation), with a = lap - c_pot (r2 - 1) psi in T, y = psi_n, v = Pi_n:
//   stage 1: acc_psi = (y + h v) + (h^2/6) a;  acc_Pi = v + (h/6) a
//            A_psi = (y + (h/2) v) + (h^2/8) a,  A_Pi = v
//   stage 2: acc_psi = acc_psi + (h^2/3) a;    acc_Pi = acc_Pi + (2h/3) a
//            B_psi = (y + h v) + (h^2/2) a,     B_Pi = v
//   stage 3: A_psi = acc_psi;  A_Pi = acc_Pi + (h/6) a   (the new U_n)
// RKN5 (stage ids 10..13; integrator type 22, read as a four-stage fifth-order Nystrom
// tableau with nodes (0, 1/5, 2/3, 1); same restrictions, single periodic levels), with
// w_ij = a_ij h^2, pb_i = bbar_i h^2, vb_i = b_i h, acc = (P, V):
//   stage 1: P = pb1 a;  V = vb1 a;  A_psi = (y + h/5 v) + w21 a;  A_Pi = S_3 = w31 a;
//            B_Pi = S_4 = w41 a
//   stage 2: P += pb2 a; V += vb2 a; B_psi = (y + 2h/3 v) + (S_3 + w32 a);  B_Pi = S_4 + w42 a
//   stage 3: P += pb3 a; V += vb3 a; A_psi = (y + h v) + (S_4 + w43 a)
//   stage 4: B_psi = (y + h v) + P;  B_Pi = v + (V + vb4 a)   (the new U_n)
// Kreiss-Oliger dissipation (KD = dissipation order 2 or 3; 0 = off) adds to the
// right-hand side of every component Q = ko * K with
//   K = (S_2 + (-4) S_1) + 18 u                    KD = 2
//     = ((S_3 + (-6) S_2) + 15 S_1) + (-60) u      KD = 3
// and ko = -eps / (16 dx) or eps / (64 dx) from the level scalars (rounded once to T):
//   k_psi = Pi + Q(psi),  k_Pi = ((lap - c_fric Pi) - c_pot (r2 - 1) psi) + Q(Pi).
// The right-hand side is evaluated in T; updates in float64, rounded to T on store.
// NT = 1 marks the streams read or written once (Pi, U_n, acc, the stage output) as
// nontemporal so they do not push the psi planes, which neighbours re-read, out of L2.
#pragma once
#include <hip/hip_runtime.h>

#include "sh_device.h"
#include "sh_internal.h"

#pragma clang fp contract(off)

// Laplacian from the per-radius neighbour sums S[r-1] and the centre value u.
template <typename T, int H>
__device__ __forceinline__ T lap_combine(const T* S, T u, T idx2) {
  if constexpr (H == 1) {
    return (S[0] - (T)6.0 * u) * idx2;
  } else if constexpr (H == 2) {
    return (((T)(4.0 / 3.0) * S[0] + (T)(-1.0 / 12.0) * S[1]) + (T)(-15.0 / 2.0) * u) * idx2;
  } else {
    static_assert(H == 3, "Laplacian orders 1, 2, 3");
    return ((((T)(3.0 / 2.0) * S[0] + (T)(-3.0 / 20.0) * S[1]) + (T)(1.0 / 90.0) * S[2]) +
            (T)(-49.0 / 6.0) * u) *
           idx2;
  }
}

// Kreiss-Oliger sum K of dissipation order KD from the neighbour sums S[r-1].
template <typename T, int KD>
__device__ __forceinline__ T ko_sum(const T* S, T u) {
  if constexpr (KD == 2) {
    return (S[1] + (T)(-4.0) * S[0]) + (T)18.0 * u;
  } else {
    static_assert(KD == 3, "dissipation orders 2, 3");
    return ((S[2] + (T)(-6.0) * S[1]) + (T)15.0 * S[0]) + (T)(-60.0) * u;
  }
}

// Six-neighbour sum at distance r read straight from memory (x, y, z).
template <typename T>
__device__ __forceinline__ T nsum(const Glob<T>* u, long long e, int r, long long px, long long plane) {
  return ((u[e - r] + u[e + r]) + (u[e - r * px] + u[e + r * px])) + (u[e - r * plane] + u[e + r * plane]);
}

template <typename T>
struct StagePtrs {
  const Glob<T>* X;
  const Glob<T>* Un;
  Glob<T>* Y;
  Glob<double>* acc;
  Glob<T>* Z;  // RKN5 stage 1: slot B, whose Pi components take the partial sum S_4
};

template <typename T, int S>
__device__ __forceinline__ StagePtrs<T> stage_ptrs(const BoxDev& B, const LevelScal& L) {
  constexpr int in_role =
      (S == 0 || S == 4 || S == 7 || S == 10) ? ROLE_UN : ((S == 2 || S == 6 || S == 9 || S == 12) ? ROLE_B : ROLE_A);
  constexpr int out_role = (S == 1 || S == 3 || S == 5 || S == 8 || S == 11 || S == 13) ? ROLE_B : ROLE_A;
  StagePtrs<T> p;
  p.X = (const Glob<T>*)slot_base(B, role_slot(in_role, L));
  p.Un = (const Glob<T>*)slot_base(B, role_slot(ROLE_UN, L));
  p.Y = (Glob<T>*)slot_base(B, role_slot(out_role, L));
  p.acc = (Glob<double>*)B.acc;
  p.Z = S == 10 ? (Glob<T>*)slot_base(B, role_slot(ROLE_B, L)) : nullptr;
  return p;
}

// Per-cell right-hand side and stage update.  p0/p1 = psi at the cell, lap0/lap1 their
// Laplacians, q0/q1 = Pi at the cell (all in T); e = element index of the cell.
// With KO, ko4 holds the dissipation terms Q of the four components.
template <typename T, int S, bool NT, bool KO = false>
__device__ __forceinline__ void stage_cell(const StageScal& sc, const Glob<T>* __restrict__ Un, Glob<T>* __restrict__ Y,
                                           Glob<double>* __restrict__ acc, long long cs, long long e, T p0, T p1,
                                           T q0, T q1, T lap0, T lap1, const double* un4, const double* acc4,
                                           const T* ko4 = nullptr, Glob<T>* __restrict__ Z = nullptr) {
  const T cf = (T)sc.cf, cp = (T)sc.cp;
  const T r2 = p0 * p0 + p1 * p1;
  const T pot = cp * (r2 - (T)1.0);
  if constexpr (S >= 10) {
    // RKN5: the acceleration, then the accumulator (position sum P, velocity sum V), the
    // next stage argument and the partial sums S_3 (in the Pi components of the stage
    // state) and S_4 (those of slot B); the tableau weights times powers of h formed
    // once in float64 (numerator times the power, then the division)
    const double h = sc.h1, hh = h * h;
    const double a[2] = {(double)(lap0 - pot * p0), (double)(lap1 - pot * p1)};
    const double s_in[2] = {(double)q0, (double)q1};  // S_3 at stage 2, S_4 at stage 3
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double y = un4[c], v = un4[2 + c];
      const long long ep = c * cs + e, eq = (2 + c) * cs + e;
      if constexpr (S == 10) {
        st<NT>(acc + ep, (hh / 24.0) * a[c]);
        st<NT>(acc + eq, (h / 24.0) * a[c]);
        st<NT>(Y + ep, (T)((y + (h / 5.0) * v) + (hh / 50.0) * a[c]));
        st<NT>(Y + eq, (T)((-(hh / 27.0)) * a[c]));
        st<NT>(Z + eq, (T)(((3.0 * hh) / 10.0) * a[c]));
      } else if constexpr (S == 11) {
        const double s4 = (double)ld<NT>((const Glob<T>*)(Y + eq));
        st<NT>(acc + ep, acc4[c] + ((25.0 * hh) / 84.0) * a[c]);
        st<NT>(acc + eq, acc4[2 + c] + ((125.0 * h) / 336.0) * a[c]);
        st<NT>(Y + ep, (T)((y + ((2.0 * h) / 3.0) * v) + (s_in[c] + ((7.0 * hh) / 27.0) * a[c])));
        st<NT>(Y + eq, (T)(s4 + (-((2.0 * hh) / 35.0)) * a[c]));
      } else if constexpr (S == 12) {
        st<NT>(acc + ep, acc4[c] + ((9.0 * hh) / 56.0) * a[c]);
        st<NT>(acc + eq, acc4[2 + c] + ((27.0 * h) / 56.0) * a[c]);
        st<NT>(Y + ep, (T)((y + h * v) + (s_in[c] + ((9.0 * hh) / 35.0) * a[c])));
      } else {
        st<NT>(Y + ep, (T)((y + h * v) + acc4[c]));
        st<NT>(Y + eq, (T)(v + (acc4[2 + c] + ((5.0 * h) / 48.0) * a[c])));
      }
    }
    return;
  } else if constexpr (S >= 7) {
    // RKN4: the acceleration, then the position/velocity updates; weights times powers
    // of h formed once in float64
    const double h = sc.h1, hh = h * h;
    const double hh6 = hh / 6.0, hh3 = hh / 3.0, hh8 = hh * 0.125, hh2 = hh * 0.5;
    const double h6 = h / 6.0, h23 = (2.0 * h) / 3.0, h2 = h * 0.5;
    const double a[2] = {(double)(lap0 - pot * p0), (double)(lap1 - pot * p1)};
    // U_n: the stage input itself at stage 1, loaded at stage 2, not needed at stage 3
    double y[2] = {0.0, 0.0}, v[2] = {0.0, 0.0};
    if constexpr (S == 7) {
      y[0] = (double)p0;
      y[1] = (double)p1;
      v[0] = (double)q0;
      v[1] = (double)q1;
    } else if constexpr (S == 8) {
      y[0] = un4[0];
      y[1] = un4[1];
      v[0] = un4[2];
      v[1] = un4[3];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const long long ep = c * cs + e, eq = (2 + c) * cs + e;
      if constexpr (S == 7) {
        st<NT>(acc + ep, (y[c] + h * v[c]) + hh6 * a[c]);
        st<NT>(acc + eq, v[c] + h6 * a[c]);
        st<NT>(Y + ep, (T)((y[c] + h2 * v[c]) + hh8 * a[c]));
        st<NT>(Y + eq, (T)v[c]);
      } else if constexpr (S == 8) {
        st<NT>(acc + ep, acc4[c] + hh3 * a[c]);
        st<NT>(acc + eq, acc4[2 + c] + h23 * a[c]);
        st<NT>(Y + ep, (T)((y[c] + h * v[c]) + hh2 * a[c]));
        st<NT>(Y + eq, (T)v[c]);
      } else {
        st<NT>(Y + ep, (T)acc4[c]);
        st<NT>(Y + eq, (T)(acc4[2 + c] + h6 * a[c]));
      }
    }
    return;
  }
  T kp0 = q0, kp1 = q1;
  T kq0 = (lap0 - cf * q0) - pot * p0;
  T kq1 = (lap1 - cf * q1) - pot * p1;
  if constexpr (KO) {
    kp0 = kp0 + ko4[0];
    kp1 = kp1 + ko4[1];
    kq0 = kq0 + ko4[2];
    kq1 = kq1 + ko4[3];
  }
  const double k4[4] = {(double)kp0, (double)kp1, (double)kq0, (double)kq1};
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

// Loads of the once-read streams of a cell: U_n (RK4 stages 2, 3; SSPRK3 stages 2, 3;
// RKN4 stage 2; every RKN5 stage) and acc (RK4 stages 2-4; RKN4 stages 2, 3; RKN5 stages
// 2-4).
template <typename T, int S, bool NT>
__device__ __forceinline__ void stage_loads(const Glob<T>* __restrict__ Un, const Glob<double>* __restrict__ acc, long long cs,
                                            long long e, double* un4, double* acc4) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if constexpr (S == 1 || S == 2 || S == 5 || S == 6 || S == 8 || S >= 10) un4[c] = (double)ld<NT>(Un + c * cs + e);
    if constexpr ((S >= 1 && S <= 3) || S == 8 || S == 9 || S >= 11) acc4[c] = ld<NT>(acc + c * cs + e);
  }
}

// Wave-row kernel: one wavefront per tile (a TX x 64/TX footprint of a box, marching
// in z); psi of planes z-HR..z+HR of both components stay in registers (HR = the wider
// of the Laplacian and dissipation radii), x and y neighbours are read through the
// caches.  Used for boxes narrower than 64 cells, and for every box with dissipation
// (whose Pi neighbours are read through the caches as well).
template <typename T, int S, bool NT, int H, int KD = 0>
__global__ __launch_bounds__(SH_BLOCK) void k_stage(const Tile* __restrict__ tiles, int ntiles,
                                                    const BoxDev* __restrict__ boxes) {
  constexpr int HR = H > KD ? H : KD;
  const int lane = threadIdx.x & (SH_WAVE - 1);
  // one tile per wavefront: the index is uniform over the wave, which keeps the tile and
  // box records and the storage bases in scalar registers
  const int t = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * (SH_BLOCK / SH_WAVE) +
                                               (threadIdx.x >> 6));
  if (t >= ntiles) return;
  const Tile tl = tiles[t];
  if (tl.box < 0) return;
  const BoxDev B = boxes[tl.box];
  const LevelScal L = load_level(B.ls);
  const StageScal sc = stage_scalars(L, S);
  const StagePtrs<T> P = stage_ptrs<T, S>(B, L);
  const Glob<T>* __restrict__ X = P.X;
  const Glob<T>* __restrict__ Un = P.Un;
  Glob<T>* __restrict__ Y = P.Y;

  const int tx = lane & ((1 << tl.txs) - 1);
  const int ty = lane >> tl.txs;
  const int x0 = tl.xy & 0xffff, y0 = tl.xy >> 16;
  const int z0 = tl.zz & 0xffff, zc = tl.zz >> 16;
  int x = x0 + tx, y = y0 + ty;
  const bool active = (x < B.nx) && (y < B.ny);
  // inactive lanes work on a valid cell (its neighbours stay within the ghost shell)
  x = min(x, B.nx - 1);
  y = min(y, B.ny - 1);
  const long long px = B.px;
  const long long plane = px * B.py;
  const long long cs = B.cs;
  const int zend = min(z0 + zc, B.nz);
  const T idx2 = (T)sc.inv_dx2;

  long long e = elem<T>(B, x, y, z0);
  // window: w[c][j] = psi_c at plane z - HR + j
  T w[2][2 * HR + 1];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int j = 0; j < 2 * HR; ++j) w[c][j] = X[c * cs + e + (j - HR) * plane];
  const T kc = (T)L.ko;
  for (int z = z0; z < zend; ++z, e += plane) {
#pragma unroll
    for (int c = 0; c < 2; ++c) w[c][2 * HR] = X[c * cs + e + HR * plane];
    T Ssum[2][HR];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const Glob<T>* u = X + c * cs;
#pragma unroll
      for (int r = 1; r <= HR; ++r)
        Ssum[c][r - 1] = ((u[e - r] + u[e + r]) + (u[e - r * px] + u[e + r * px])) + (w[c][HR - r] + w[c][HR + r]);
    }
    const T q0 = ld<NT>(X + 2 * cs + e), q1 = ld<NT>(X + 3 * cs + e);
    double un4[4], acc4[4];
    stage_loads<T, S, NT>(Un, P.acc, cs, e, un4, acc4);
    const T lap0 = lap_combine<T, H>(Ssum[0], w[0][HR], idx2);
    const T lap1 = lap_combine<T, H>(Ssum[1], w[1][HR], idx2);
    if constexpr (KD > 0) {
      T ko4[4];
      ko4[0] = kc * ko_sum<T, KD>(Ssum[0], w[0][HR]);
      ko4[1] = kc * ko_sum<T, KD>(Ssum[1], w[1][HR]);
      T Sq[2][KD];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 1; r <= KD; ++r) Sq[c][r - 1] = nsum(X + (2 + c) * cs, e, r, px, plane);
      ko4[2] = kc * ko_sum<T, KD>(Sq[0], q0);
      ko4[3] = kc * ko_sum<T, KD>(Sq[1], q1);
      if (active)
        stage_cell<T, S, NT, true>(sc, Un, Y, P.acc, cs, e, w[0][HR], w[1][HR], q0, q1, lap0, lap1, un4, acc4, ko4,
                                   P.Z);
    } else {
      if (active)
        stage_cell<T, S, NT>(sc, Un, Y, P.acc, cs, e, w[0][HR], w[1][HR], q0, q1, lap0, lap1, un4, acc4, nullptr, P.Z);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 2 * HR; ++j) w[c][j] = w[c][j + 1];
  }
}

// Block-row kernel for boxes at least 64 cells wide: a block of ROWS wavefronts covers a
// 64 x ROWS footprint (wave w owns row y0 + w) and marches in z in lock step.  Each wave
// keeps the stencilled components at planes z-HR..z+HR of its own row in registers and
// publishes plane z of the row to LDS, where the rows above and below (and the HR x-halo
// columns on each side, loaded by the edge lanes; the HR halo rows on each side, loaded
// by the first and last waves) are read back.  The stencilled components are psi (the
// Laplacian, radius H) and, with dissipation (order KD), Pi as well; HR is the wider
// radius.  Each is therefore fetched about (ROWS+2HR)/ROWS times per plane instead of
// 4HR+1 times through the caches.
template <typename T, int S, bool NT, int ROWS, int H, int KD = 0>
__global__ __launch_bounds__(SH_WAVE * ROWS) void k_stage_lds(const Tile* __restrict__ tiles, int ntiles,
                                                              const BoxDev* __restrict__ boxes) {
  constexpr int HR = H > KD ? H : KD;  // halo radius
  constexpr int NC = KD > 0 ? 4 : 2;   // stencilled components
  static_assert(HR <= ROWS && HR < SH_WAVE / 2, "halo loads by the edge waves and lanes");
  __shared__ T sm[2][NC][ROWS + 2 * HR][SH_WAVE + 2 * HR];
  const int lane = threadIdx.x & (SH_WAVE - 1);
  const int w = threadIdx.x >> 6;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  if (t >= ntiles) return;  // uniform over the block
  const Tile tl = tiles[t];
  if (tl.box < 0) return;
  const BoxDev B = boxes[tl.box];
  const LevelScal L = load_level(B.ls);
  const StageScal sc = stage_scalars(L, S);
  const StagePtrs<T> P = stage_ptrs<T, S>(B, L);
  const Glob<T>* __restrict__ X = P.X;
  const Glob<T>* __restrict__ Un = P.Un;
  Glob<T>* __restrict__ Y = P.Y;

  const int x0 = tl.xy & 0xffff, y0 = tl.xy >> 16;
  const int z0 = tl.zz & 0xffff, zc = tl.zz >> 16;
  const int x = x0 + lane, y = y0 + w;
  const bool active = (x < B.nx) && (y < B.ny);
  // rows and columns past the box edge load the ghost rows/columns instead (valid
  // memory: the shell is at least HR deep), so the active cells next to the edge read
  // their true neighbours from LDS
  const int xl = min(x, B.nx + HR - 1), yl = min(y, B.ny + HR - 1);
  const long long px = B.px;
  const long long plane = px * B.py;
  const long long cs = B.cs;
  const int zend = min(z0 + zc, B.nz);
  const T idx2 = (T)sc.inv_dx2;
  const T kc = (T)L.ko;

  long long e = elem<T>(B, xl, yl, z0);
  // halo rows: waves 0..HR-1 load rows y0-HR.., waves ROWS-HR.. load rows y0+ROWS..; when
  // the two sets are disjoint (ROWS >= 2HR) a wave holds one halo row (one address, one
  // value per component), else the middle waves hold two
  constexpr bool ONE_H = ROWS >= 2 * HR;
  const bool has_lo = w < HR, has_hi = w >= ROWS - HR;
  const long long elo = elem<T>(B, xl, has_lo ? y0 - HR + w : yl, z0);
  const long long ehi = elem<T>(B, xl, has_hi ? min(y0 + ROWS + w - (ROWS - HR), B.ny + HR - 1) : yl, z0);
  const long long eh1 = has_lo ? elo : ehi;  // ONE_H: the wave's halo row
  const int hrow1 = has_lo ? w : w + 2 * HR;
  // x-halo columns: lanes 0..HR-1 load x0-HR.., lanes 64-HR.. load x0+64.. (disjoint sets)
  const bool has_x = lane < HR || lane >= SH_WAVE - HR;
  const long long ex = elem<T>(B, lane < HR ? x0 - HR + lane : min(x0 + lane + HR, B.nx + HR - 1), yl, z0);
  const int xcol = lane < HR ? lane : lane + 2 * HR;

  T win[NC][2 * HR + 1];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int j = 0; j < 2 * HR; ++j) win[c][j] = X[c * cs + e + (j - HR) * plane];
  int buf = 0;
  for (int z = z0; z < zend; ++z, e += plane, buf ^= 1) {
    const long long zo = (long long)(z - z0) * plane;
    T hlo[NC], hhi[NC], vx[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      hlo[c] = hhi[c] = vx[c] = (T)0;
      win[c][2 * HR] = X[c * cs + e + HR * plane];
      if constexpr (ONE_H) {
        if (has_lo || has_hi) hlo[c] = X[c * cs + eh1 + zo];
      } else {
        if (has_lo) hlo[c] = X[c * cs + elo + zo];
        if (has_hi) hhi[c] = X[c * cs + ehi + zo];
      }
      if (has_x) vx[c] = X[c * cs + ex + zo];
    }
    T q0, q1;
    if constexpr (KD > 0) {
      q0 = win[2][HR];
      q1 = win[3][HR];
    } else {
      q0 = ld<NT>(X + 2 * cs + e);
      q1 = ld<NT>(X + 3 * cs + e);
    }
    double un4[4], acc4[4];
    stage_loads<T, S, NT>(Un, P.acc, cs, e, un4, acc4);
    // LDS row j holds y = y0 - HR + j, column i holds x = x0 - HR + i
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      sm[buf][c][w + HR][lane + HR] = win[c][HR];
      if constexpr (ONE_H) {
        if (has_lo || has_hi) sm[buf][c][hrow1][lane + HR] = hlo[c];
      } else {
        if (has_lo) sm[buf][c][w][lane + HR] = hlo[c];
        if (has_hi) sm[buf][c][w + 2 * HR][lane + HR] = hhi[c];
      }
      if (has_x) sm[buf][c][w + HR][xcol] = vx[c];
    }
    lds_barrier();
    // per-radius neighbour sums of every stencilled component (Laplacian: psi, radii
    // 1..H; dissipation: every component, radii 1..KD), used up one component at a time
    T lapc[2], ko4[4];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T Ssum[HR];
#pragma unroll
      for (int r = 1; r <= HR; ++r) {
        const T xm = sm[buf][c][w + HR][lane + HR - r], xp = sm[buf][c][w + HR][lane + HR + r];
        const T ym = sm[buf][c][w + HR - r][lane + HR], yp = sm[buf][c][w + HR + r][lane + HR];
        Ssum[r - 1] = ((xm + xp) + (ym + yp)) + (win[c][HR - r] + win[c][HR + r]);
      }
      if (c < 2) lapc[c] = lap_combine<T, H>(Ssum, win[c][HR], idx2);
      if constexpr (KD > 0) ko4[c] = kc * ko_sum<T, KD>(Ssum, win[c][HR]);
    }
    const T lap0 = lapc[0], lap1 = lapc[1];
    if constexpr (KD > 0) {
      if (active)
        stage_cell<T, S, NT, true>(sc, Un, Y, P.acc, cs, e, win[0][HR], win[1][HR], q0, q1, lap0, lap1, un4, acc4,
                                   ko4);
    } else {
      if (active)
        stage_cell<T, S, NT>(sc, Un, Y, P.acc, cs, e, win[0][HR], win[1][HR], q0, q1, lap0, lap1, un4, acc4, nullptr,
                             P.Z);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int j = 0; j < 2 * HR; ++j) win[c][j] = win[c][j + 1];
  }
}

// Right-hand side only (diagnostic): out[box][c][z][y][x] = f(U_n) at stage-1 scalars.
template <typename T, int H, int KD = 0>
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
  const LevelScal L = load_level(B.ls);
  const StageScal sc = stage_scalars(L, 0);
  const Glob<T>* __restrict__ X = (const Glob<T>*)slot_base(B, role_slot(ROLE_UN, L));
  const int tx = lane & ((1 << tl.txs) - 1), ty = lane >> tl.txs;
  const int x = (tl.xy & 0xffff) + tx, y = (tl.xy >> 16) + ty;
  if (x >= B.nx || y >= B.ny) return;
  const int z0 = tl.zz & 0xffff, zend = min(z0 + (tl.zz >> 16), B.nz);
  const long long px = B.px, plane = px * B.py, cs = B.cs;
  const long long nv = (long long)B.nx * B.ny * B.nz;
  const T cf = (T)sc.cf, cp = (T)sc.cp, idx2 = (T)sc.inv_dx2;
  constexpr int HR = H > KD ? H : KD;
  const T kc = (T)L.ko;
  for (int z = z0; z < zend; ++z) {
    const long long e = elem<T>(B, x, y, z);
    T lap[2], ko4[4] = {(T)0, (T)0, (T)0, (T)0};
    for (int c = 0; c < 2; ++c) {
      const Glob<T>* u = X + c * cs;
      T Ssum[HR];
#pragma unroll
      for (int r = 1; r <= HR; ++r) Ssum[r - 1] = nsum(u, e, r, px, plane);
      lap[c] = lap_combine<T, H>(Ssum, u[e], idx2);
      if constexpr (KD > 0) ko4[c] = kc * ko_sum<T, KD>(Ssum, u[e]);
    }
    const T p0 = X[e], p1 = X[cs + e], q0 = X[2 * cs + e], q1 = X[3 * cs + e];
    if constexpr (KD > 0) {
      for (int c = 0; c < 2; ++c) {
        T Sq[KD];
#pragma unroll
        for (int r = 1; r <= KD; ++r) Sq[r - 1] = nsum(X + (2 + c) * cs, e, r, px, plane);
        ko4[2 + c] = kc * ko_sum<T, KD>(Sq, c == 0 ? q0 : q1);
      }
    }
    const T r2 = p0 * p0 + p1 * p1;
    const T pot = cp * (r2 - (T)1.0);
    const long long o = out_off[tl.box] + ((long long)z * B.ny + y) * B.nx + x;
    T kp0 = q0, kp1 = q1, kq0 = (lap[0] - cf * q0) - pot * p0, kq1 = (lap[1] - cf * q1) - pot * p1;
    if constexpr (KD > 0) {
      kp0 = kp0 + ko4[0];
      kp1 = kp1 + ko4[1];
      kq0 = kq0 + ko4[2];
      kq1 = kq1 + ko4[3];
    }
    out[o] = (double)kp0;
    out[o + nv] = (double)kp1;
    out[o + 2 * nv] = (double)kq0;
    out[o + 3 * nv] = (double)kq1;
  }
}

// ---------------------------------------------------------------------------------
// Host-side launch of one stage (kind: 0 = wave-row tiles, 4 or 8 = block-row tiles of
// that many rows) and of the diagnostic right-hand side, for stencil radius H.
// ---------------------------------------------------------------------------------
template <typename T, int S, bool NT, int H>
static void stage_launch3(int kind, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  if (ntiles == 0) return;
  if (kind == 0) {
    hipLaunchKernelGGL((k_stage<T, S, NT, H>), dim3((ntiles + SH_BLOCK / SH_WAVE - 1) / (SH_BLOCK / SH_WAVE)),
                       dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes);
  } else if (kind == 4) {
    hipLaunchKernelGGL((k_stage_lds<T, S, NT, 4, H>), dim3(ntiles), dim3(SH_WAVE * 4), 0, st, tiles, ntiles, boxes);
  } else {
    hipLaunchKernelGGL((k_stage_lds<T, S, NT, 8, H>), dim3(ntiles), dim3(SH_WAVE * 8), 0, st, tiles, ntiles, boxes);
  }
}

template <typename T, bool NT, int H>
static void stage_launch2(int s, int kind, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  switch (s) {
    case 0: stage_launch3<T, 0, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 1: stage_launch3<T, 1, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 2: stage_launch3<T, 2, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 3: stage_launch3<T, 3, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 4: stage_launch3<T, 4, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 5: stage_launch3<T, 5, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 6: stage_launch3<T, 6, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 7: stage_launch3<T, 7, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 8: stage_launch3<T, 8, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 9: stage_launch3<T, 9, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 10: stage_launch3<T, 10, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 11: stage_launch3<T, 11, NT, H>(kind, tiles, ntiles, boxes, st); break;
    case 12: stage_launch3<T, 12, NT, H>(kind, tiles, ntiles, boxes, st); break;
    default: stage_launch3<T, 13, NT, H>(kind, tiles, ntiles, boxes, st); break;
  }
}

template <int H>
static void stage_launch_radius(int prec, int s, int kind, bool nt, const Tile* tiles, int ntiles,
                                const BoxDev* boxes, hipStream_t st) {
  if (prec == 0) {
    if (nt) stage_launch2<double, true, H>(s, kind, tiles, ntiles, boxes, st);
    else stage_launch2<double, false, H>(s, kind, tiles, ntiles, boxes, st);
  } else {
    if (nt) stage_launch2<float, true, H>(s, kind, tiles, ntiles, boxes, st);
    else stage_launch2<float, false, H>(s, kind, tiles, ntiles, boxes, st);
  }
}

template <int H>
static void rhs_launch_radius(int prec, const Tile* tiles, int ntiles, const BoxDev* boxes, const long long* out_off,
                              double* out, hipStream_t st) {
  const int nb = (ntiles + SH_BLOCK / SH_WAVE - 1) / (SH_BLOCK / SH_WAVE);
  if (nb == 0) return;
  if (prec == 0) hipLaunchKernelGGL((k_rhs<double, H>), dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, out_off, out);
  else hipLaunchKernelGGL((k_rhs<float, H>), dim3(nb), dim3(SH_BLOCK), 0, st, tiles, ntiles, boxes, out_off, out);
}
