// Fused step: all NS stages of a step in one kernel (temporal blocking), for classic RK4
// (NS = 4) and SSPRK3 (NS = 3).
//
// The arithmetic is exactly that of the per-stage kernel (same expressions, same order,
// stage states rounded to the storage type between stages), so the results are the same
// bit for bit; only the data movement changes.  The per-stage form moves 64 (RK4: U_n,
// stage states and the accumulator, 12/20/20/12 per stage) or 32 (SSPRK3: 8/12/12)
// values per cell and step through HBM; fused, each step reads U_n and writes U_{n+1}
// once: 8 values per cell.
//
// Scheme.  A block owns a TX x TY column footprint of a box and marches up a range of zc
// planes.  Stage j (0..NS-1) of plane p runs in iteration p + j, after stage j-1 of plane
// p+1 (its z+1 neighbour) in the same iteration, so each stage keeps a three-plane
// window of its input column in registers.  In x and y a stage needs its input one cell
// beyond where it is computed, so stage j is computed on the footprint grown by
// NS - 1 - j cells (overlapped tiles), and the threads cover the footprint grown by NS
// cells, the outermost ring only loading U_n.  Each iteration every stage publishes its
// input plane to LDS, a barrier, the stages run in order reading x/y neighbours from LDS,
// and a second barrier closes the iteration.  (Two plane buffers alternating by
// iteration, which need only the first barrier and can also serve the z-1 neighbour of
// stages 1..3, measured slower in every variant and precision at 512^3: 5-25 %.)
// The z-range is extended the same way (stage j covers NS - 1 - j extra planes below and
// above), so U_n is read from z0-NS to z0+zc+NS-1: the level keeps a 4-deep ghost shell.
// The RK4 accumulator exists only on the footprint's own columns (registers or LDS).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "sh_device.h"
#include "sh_internal.h"
#include "sh_launch.h"

#pragma clang fp contract(off)

namespace {

// FD = NS fused stages; stage 0 is computed on the footprint grown by FG = FD - 1 cells
template <typename T, int TX, int TY, int FD>
struct FusedShape {
  static constexpr int W = TX + 2 * FD;  // thread columns in x (incl. the loader ring)
  static constexpr int H = TY + 2 * FD;
  static constexpr int NTH = W * H;
  static constexpr int NBLK = (NTH + SH_WAVE - 1) / SH_WAVE * SH_WAVE;
};

// Thread -> column map sorted by ring distance from the footprint (footprint first, then
// rings 1..FD), row-major within a ring.  Stage j is computed on rings 0..FG-j, so with
// this order whole wavefronts skip the stages they have no columns for.
template <int TX, int TY, int FD>
struct RingMap {
  static constexpr int W = TX + 2 * FD, H = TY + 2 * FD, N = W * H;
  unsigned char cx[N], cy[N];
  constexpr RingMap() : cx(), cy() {
    int k = 0;
    for (int r = 0; r <= FD; ++r)
      for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
          const int ox = x - FD, oy = y - FD;
          const int rx = ox < 0 ? -ox : (ox >= TX ? ox - TX + 1 : 0);
          const int ry = oy < 0 ? -oy : (oy >= TY ? oy - TY + 1 : 0);
          if ((rx > ry ? rx : ry) == r) {
            cx[k] = (unsigned char)x;
            cy[k] = (unsigned char)y;
            ++k;
          }
        }
  }
};

template <int TX, int TY, int FD>
__constant__ RingMap<TX, TY, FD> ring_map = RingMap<TX, TY, FD>();

}  // namespace

// DPP lane shifts (GFX9 wavefront shift by one lane; lane 0 / 63 receive `old`).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v, double old) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v, float old) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane l takes lane l-1
constexpr int DPP_WAVE_SHL1 = 0x130;  // lane l takes lane l+1

// NS: 4 = classic RK4, 3 = SSPRK3 (stage updates as in the per-stage kernel).
// ORDER 0: threads row-major over the (TX+2NS) x (TY+2NS) columns; 1: sorted by ring.
// XDPP: x neighbours by lane shifts (row-major only: the computing columns' x neighbours
// are the adjacent lanes; the two wave-edge lanes read LDS).  ACCL: RK4 accumulator in
// LDS.
// PF2: U_n planes are loaded two iterations before they enter the stage-0 window, into
// two buffers that alternate between iterations (else in the iteration that uses them).
// UNG: the U_n values the updates of stages 1 and 2 need (planes i-1 and i-2, read two and
// one iterations earlier by the same thread, so still in the caches) are read again from
// memory instead of being carried in registers.
template <typename T, bool NT, int TX, int TY, int ORDER, bool XDPP, bool ACCL, bool PF2, int NS,
          bool UNG = false>
__global__ __launch_bounds__((FusedShape<T, TX, TY, NS>::NBLK)) void k_fused_step(const Tile* __restrict__ tiles,
                                                                                int ntiles,
                                                                                const BoxDev* __restrict__ boxes) {
  static_assert(!(XDPP && ORDER != 0), "lane shifts need the row-major order");
  static_assert(NS == 4 || (NS == 3 && !ACCL), "RK4 (with either accumulator) or SSPRK3 (none)");
  constexpr int FD = NS;      // fused stages
  constexpr int FG = FD - 1;  // compute ring of stage 0 beyond the footprint
  using Sh = FusedShape<T, TX, TY, FD>;
  constexpr int W = Sh::W, H = Sh::H;
  // stage input planes (psi of both components); every write of an iteration comes after
  // the previous iteration's closing barrier, every read before this one's
  __shared__ T sm[FD][2][H][W];
  // RK4 accumulator of the footprint's own columns for the four planes in flight (slot =
  // plane mod 4); each thread touches only its own column, so no barrier is involved
  __shared__ double sacc[ACCL ? 4 : 1][4][ACCL ? TY : 1][ACCL ? TX : 1];

  const int t = xcd_remap(blockIdx.x, gridDim.x);
  if (t >= ntiles) return;  // uniform
  const Tile tl = tiles[t];
  if (tl.box < 0) return;
  const BoxDev B = boxes[tl.box];
  const LevelScal L = *B.ls;
  StageScal sc[FD];
#pragma unroll
  for (int j = 0; j < FD; ++j) sc[j] = uniform(stage_scalars(L, NS == 4 ? j : j + 4));
  // U_n in, U_{n+1} out: RK4's last stage writes B, SSPRK3's writes A (the role cycle of
  // the integrator, which the launch matches)
  const T* __restrict__ X = (const T*)slot_base(B, role_slot(ROLE_UN, L.k, NS));
  T* __restrict__ Y = (T*)slot_base(B, role_slot(NS == 4 ? ROLE_B : ROLE_A, L.k, NS));

  const int tid = threadIdx.x;
  const int lane = tid & (SH_WAVE - 1);
  const bool inreg = tid < Sh::NTH;
  int cx = FD, cy = FD;
  if (inreg) {
    if (ORDER == 0) {
      cx = tid % W;
      cy = tid / W;
    } else {
      cx = ring_map<TX, TY, FD>.cx[tid];
      cy = ring_map<TX, TY, FD>.cy[tid];
    }
  }
  const int ox = cx - FD, oy = cy - FD;  // footprint-relative
  const int rx = ox < 0 ? -ox : (ox >= TX ? ox - TX + 1 : 0);
  const int ry = oy < 0 ? -oy : (oy >= TY ? oy - TY + 1 : 0);
  const int r = inreg ? max(rx, ry) : FD + 1;  // ring distance; > FD: idle thread
  const int x0 = tl.xy & 0xffff, y0 = tl.xy >> 16;
  const int z0 = tl.zz & 0xffff, zc = tl.zz >> 16;
  // footprints tile the box exactly and the ghost shell is FD deep: every column a
  // thread loads lies in [-FD, n + FD); idle threads load the footprint's first column
  const int x = x0 + (r <= FD ? ox : 0), y = y0 + (r <= FD ? oy : 0);
  const long long plane = (long long)B.px * B.py;
  const long long cs = B.cs;
  // this thread's column of U_n (psi1, psi2, Pi1, Pi2) and of the output, at plane 0
  typedef __attribute__((address_space(1))) const T* gcptr;
  typedef __attribute__((address_space(1))) T* gptr;
  gcptr col = (gcptr)(X + elem<T>(B, x, y, 0));
  gptr ocol = (gptr)(Y + elem<T>(B, x, y, 0));
  const int zlo = -B.ng, zhi = B.nz + B.ng - 1;
  auto eat = [&](int z) { return (long long)min(max(z, zlo), zhi) * plane; };

  const int ifirst = z0 - FG, ilast = z0 + zc - 1 + FG;
  // stage 0 input window (planes i-1, i, i+1) and Pi of plane i
  T w0[3][2], q0c[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    w0[0][c] = col[c * cs + eat(ifirst - 1)];
    w0[1][c] = col[c * cs + eat(ifirst)];
    w0[2][c] = col[c * cs + eat(ifirst + 1)];
    q0c[c] = (r <= FG) ? col[(2 + c) * cs + eat(ifirst)] : (T)0;
  }
  // later stages: input windows and their Pi at planes (p, p+1); U_n at planes i-1, i-2
  // (psi of i-1 is the window bottom) for the updates of stages 1 and 2
  T wj[FD][3][2], qj[FD][2][2];
  T q0p[2] = {(T)0, (T)0}, u2[4] = {(T)0, (T)0, (T)0, (T)0};
  double racc[NS == 4 ? FD : 1][4];
#pragma unroll
  for (int j = 0; j < FD; ++j) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      wj[j][0][c] = wj[j][1][c] = wj[j][2][c] = (T)0;
      qj[j][0][c] = qj[j][1][c] = (T)0;
    }
    if constexpr (NS == 4) {
#pragma unroll
      for (int c = 0; c < 4; ++c) racc[j][c] = 0.0;
    }
  }
  const bool own = (r == 0);
  const int ax = own ? ox : 0, ay = own ? oy : 0;
  const bool edge_lane = (lane == 0) || (lane == SH_WAVE - 1);
  const int cxm = max(cx - 1, 0), cxp = min(cx + 1, W - 1);
  const int cym = max(cy - 1, 0), cyp = min(cy + 1, H - 1);

  // one iteration: stage j handles plane i - j.  FILL marks the first 2*FG iterations,
  // in which the later stages are still waiting for their input windows to fill.
  // U_n planes on their way into the stage-0 window: [psi / Pi][component].  Loads are
  // issued at the top of an iteration; without PF2 they enter the window at its end, with
  // PF2 at the end of the next one.  A value still in flight is never copied between
  // registers (that would wait for it at the loop's back edge), so with PF2 the two
  // buffers swap roles from one iteration to the next instead.
  T pfa[2][2], pfb[2][2];
  auto load_planes = [&](const int zpsi, T(&dst)[2][2]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      dst[0][c] = col[c * cs + eat(zpsi)];
      // Pi only where stage 0 is computed: the outer loader ring supplies psi alone
      dst[1][c] = (r <= FG) ? col[(2 + c) * cs + eat(zpsi - 1)] : (T)0;
    }
  };
  auto iteration = [&](const int i, auto fill_tag, T(&ldb)[2][2], T(&useb)[2][2]) {
    constexpr bool FILL = decltype(fill_tag)::value;
    load_planes(PF2 ? i + 3 : i + 2, ldb);
    // publish every stage's input plane: stage 0 = U_n psi at i, stage j = its window top
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (r <= FD) sm[0][c][cy][cx] = w0[1][c];
#pragma unroll
      for (int j = 1; j < FD; ++j)
        if (r <= FD - j) sm[j][c][cy][cx] = wj[j][2][c];
    }
    lds_barrier();
    // outputs of the stage just computed (input of the next one)
    T out[4];
#pragma unroll
    for (int j = 0; j < FD; ++j) {
      // stage j runs from iteration ifirst + 2j on; before that its window fills with the
      // planes stage j-1 produces (the conditions are uniform over the block)
      if (j > 0) {
        if (FILL && i < ifirst + 2 * (j - 1)) break;
        // push stage j-1's output plane (p+1) into stage j's window
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          wj[j][0][c] = wj[j][1][c];
          wj[j][1][c] = wj[j][2][c];
          wj[j][2][c] = out[c];
          qj[j][0][c] = qj[j][1][c];
          qj[j][1][c] = out[2 + c];
        }
      }
      if (FILL && i < ifirst + 2 * j) break;
      T(*w)[2] = (j == 0) ? w0 : wj[j];
      // x neighbours by lane shifts: done with every lane active (before the ring test)
      T xs[2][2];
      if (XDPP) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          xs[c][0] = dpp_move<DPP_WAVE_SHR1>(w[1][c], w[1][c]);
          xs[c][1] = dpp_move<DPP_WAVE_SHL1>(w[1][c], w[1][c]);
        }
      }
      if (r > FG - j) continue;
      const T q0 = (j == 0) ? q0c[0] : qj[j][0][0];
      const T q1 = (j == 0) ? q0c[1] : qj[j][0][1];
      const T idx2 = (T)sc[j].inv_dx2, cf = (T)sc[j].cf, cp = (T)sc[j].cp;
      T lap[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T xm, xp;
        if (XDPP) {
          xm = xs[c][0];
          xp = xs[c][1];
          if (edge_lane) {
            xm = sm[j][c][cy][cxm];
            xp = sm[j][c][cy][cxp];
          }
        } else {
          xm = sm[j][c][cy][cx - 1];
          xp = sm[j][c][cy][cx + 1];
        }
        const T ym = sm[j][c][cym][cx], yp = sm[j][c][cyp][cx];
        const T zm = w[0][c];
        lap[c] = ((((xm + xp) + (ym + yp)) + (zm + w[2][c])) - (T)6.0 * w[1][c]) * idx2;
      }
      const T p0 = w[1][0], p1 = w[1][1];
      const T r2 = p0 * p0 + p1 * p1;
      const T pot = cp * (r2 - (T)1.0);
      const T kq0 = (lap[0] - cf * q0) - pot * p0;
      const T kq1 = (lap[1] - cf * q1) - pot * p1;
      const double k4[4] = {(double)q0, (double)q1, (double)kq0, (double)kq1};
      const T xin[4] = {p0, p1, q0, q1};
      // U_n at the stage's plane (stage 1: plane i-1, stage 2: plane i-2)
      T un[4] = {(T)0, (T)0, (T)0, (T)0};
      if (j == 1) {
        un[0] = w0[0][0];
        un[1] = w0[0][1];
        un[2] = UNG ? col[2 * cs + eat(i - 1)] : q0p[0];
        un[3] = UNG ? col[3 * cs + eat(i - 1)] : q0p[1];
      } else if (j == 2) {
#pragma unroll
        for (int c = 0; c < 4; ++c) un[c] = UNG ? col[c * cs + eat(i - 2)] : u2[c];
      }
      constexpr int AST = ACCL ? TY * TX : 1;  // component stride of sacc
      double* ac = ACCL ? &sacc[(i - j) & 3][0][ay][ax] : &racc[NS == 4 ? j : 0][0];
      const int ast = ACCL ? AST : 1;
      // the LDS accumulator exists for the footprint's columns only; the register one is
      // updated on every computing column (values off the footprint are never stored)
      const bool upd = ACCL ? own : true;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if constexpr (NS == 3) {
          // SSPRK3: U_n + h k;  3/4 U_n + 1/4 (X + h k);  1/3 U_n + 2/3 (X + h k)
          const double xk = (double)xin[c] + sc[j].h1 * k4[c];
          if (j == 0) out[c] = (T)xk;
          else if (j == 1) out[c] = (T)(0.75 * (double)un[c] + 0.25 * xk);
          else out[c] = (T)((1.0 / 3.0) * (double)un[c] + (2.0 / 3.0) * xk);
        } else if (j == 0) {
          const double u = (double)xin[c];
          if (upd) ac[c * ast] = u + sc[0].h6 * k4[c];
          out[c] = (T)(u + sc[0].h2 * k4[c]);
        } else if (j == 1) {
          if (upd) ac[c * ast] = ac[c * ast] + sc[1].h3 * k4[c];
          out[c] = (T)((double)un[c] + sc[1].h2 * k4[c]);
        } else if (j == 2) {
          if (upd) ac[c * ast] = ac[c * ast] + sc[2].h3 * k4[c];
          out[c] = (T)((double)un[c] + sc[2].h1 * k4[c]);
        } else {
          out[c] = (T)(ac[c * ast] + sc[3].h6 * k4[c]);
        }
      }
      if (j == FD - 1 && own) {
        const long long e = (long long)(i - FG) * plane;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if constexpr (NT) __builtin_nontemporal_store(out[c], ocol + c * cs + e);
          else ocol[c * cs + e] = out[c];
        }
      }
    }
    lds_barrier();
    if constexpr (NS == 4 && !ACCL) {
      // register accumulator: advance the per-plane chain by one plane
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = FD - 1; j > 0; --j) racc[j][c] = racc[j - 1][c];
    }
    // advance the stage-0 window by one plane
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      u2[c] = w0[0][c];
      u2[2 + c] = q0p[c];
      w0[0][c] = w0[1][c];
      w0[1][c] = w0[2][c];
      w0[2][c] = useb[0][c];
      q0p[c] = q0c[c];
      q0c[c] = useb[1][c];
    }
  };
  // every tile has zc + 2 FG >= 2 FG + 1 iterations: the filling ones (an even number)
  // always run in full
  int i = ifirst;
  if constexpr (PF2) {
    load_planes(ifirst + 2, pfb);
    for (; i < ifirst + 2 * FG; i += 2) {
      iteration(i, std::true_type{}, pfa, pfb);
      iteration(i + 1, std::true_type{}, pfb, pfa);
    }
    for (; i + 1 <= ilast; i += 2) {
      iteration(i, std::false_type{}, pfa, pfb);
      iteration(i + 1, std::false_type{}, pfb, pfa);
    }
    if (i <= ilast) iteration(i, std::false_type{}, pfa, pfb);
  } else {
    for (; i < ifirst + 2 * FG; ++i) iteration(i, std::true_type{}, pfa, pfa);
    for (; i <= ilast; ++i) iteration(i, std::false_type{}, pfa, pfa);
  }
}

template <typename T, bool NT, int TX, int TY, int NS, int ORDER, bool XDPP, bool ACCL, bool PF2 = false,
          bool UNG = false>
static void fused_launch_shape(const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  using Sh = FusedShape<T, TX, TY, NS>;
  hipLaunchKernelGGL((k_fused_step<T, NT, TX, TY, ORDER, XDPP, ACCL, PF2, NS, UNG>), dim3(ntiles), dim3(Sh::NBLK),
                     0, st, tiles, ntiles, boxes);
}

// variant: 0 = row-major threads, x neighbours through LDS, accumulator in registers;
// 1 = row-major, x neighbours by lane shifts, registers; 2 = row-major, lane shifts,
// accumulator in LDS; 3 = ring-ordered threads, LDS neighbours, accumulator in LDS;
// 4 = ring-ordered threads, LDS neighbours, accumulator in registers; 5 = variant 4 with
// the two-iteration U_n prefetch; 6 = variant 5 with the accumulator in LDS; 7 =
// ring-ordered threads, accumulator in LDS, U_n of stages 1 and 2 read again from memory
// (fewer registers); 8 = variant 7 with the two-iteration U_n prefetch.  SSPRK3 has no
// accumulator: variants 2, 3 and 6 run as 1, 4 and 5, and 7 and 8 keep only the re-read
// of U_n.
template <typename T, bool NT, int TX, int TY, int NS>
static void fused_launch_variant(int variant, const Tile* tiles, int ntiles, const BoxDev* boxes, hipStream_t st) {
  constexpr bool AL = NS == 4;  // the LDS accumulator variants exist for RK4
  switch (variant) {
    case 0: fused_launch_shape<T, NT, TX, TY, NS, 0, false, false>(tiles, ntiles, boxes, st); break;
    case 1: fused_launch_shape<T, NT, TX, TY, NS, 0, true, false>(tiles, ntiles, boxes, st); break;
    case 2: fused_launch_shape<T, NT, TX, TY, NS, 0, true, AL>(tiles, ntiles, boxes, st); break;
    case 3: fused_launch_shape<T, NT, TX, TY, NS, 1, false, AL>(tiles, ntiles, boxes, st); break;
    case 4: fused_launch_shape<T, NT, TX, TY, NS, 1, false, false>(tiles, ntiles, boxes, st); break;
    case 5: fused_launch_shape<T, NT, TX, TY, NS, 1, false, false, true>(tiles, ntiles, boxes, st); break;
    case 6: fused_launch_shape<T, NT, TX, TY, NS, 1, false, AL, true>(tiles, ntiles, boxes, st); break;
    case 7: fused_launch_shape<T, NT, TX, TY, NS, 1, false, AL, false, true>(tiles, ntiles, boxes, st); break;
    default: fused_launch_shape<T, NT, TX, TY, NS, 1, false, AL, true, true>(tiles, ntiles, boxes, st); break;
  }
}

template <typename T, bool NT, int NS>
static void fused_launch(int shape, int variant, const Tile* tiles, int ntiles, const BoxDev* boxes,
                         hipStream_t st) {
  if (ntiles == 0) return;
  if (shape == 0) fused_launch_variant<T, NT, 32, 8, NS>(variant, tiles, ntiles, boxes, st);
  else if (shape == 1) fused_launch_variant<T, NT, 64, 4, NS>(variant, tiles, ntiles, boxes, st);
  else if (shape == 2) fused_launch_variant<T, NT, 32, 16, NS>(variant, tiles, ntiles, boxes, st);
  else fused_launch_variant<T, NT, 16, 8, NS>(variant, tiles, ntiles, boxes, st);
}

// Footprint of a fused tile: shape 0 = 32 x 8, 1 = 64 x 4, 2 = 32 x 16, 3 = 16 x 8 (two
// workgroups per CU).
void sh_fused_footprint(int shape, int* tx, int* ty) {
  static const int fx[4] = {32, 64, 32, 16}, fy[4] = {8, 4, 16, 8};
  *tx = fx[shape];
  *ty = fy[shape];
}

void sh_launch_fused(int prec, bool nt, int shape, int variant, int nst, const Tile* tiles, int ntiles,
                     const BoxDev* boxes, hipStream_t st) {
  if (nst == 3) {
    if (prec == 0) {
      if (nt) fused_launch<double, true, 3>(shape, variant, tiles, ntiles, boxes, st);
      else fused_launch<double, false, 3>(shape, variant, tiles, ntiles, boxes, st);
    } else {
      if (nt) fused_launch<float, true, 3>(shape, variant, tiles, ntiles, boxes, st);
      else fused_launch<float, false, 3>(shape, variant, tiles, ntiles, boxes, st);
    }
  } else if (prec == 0) {
    if (nt) fused_launch<double, true, 4>(shape, variant, tiles, ntiles, boxes, st);
    else fused_launch<double, false, 4>(shape, variant, tiles, ntiles, boxes, st);
  } else {
    if (nt) fused_launch<float, true, 4>(shape, variant, tiles, ntiles, boxes, st);
    else fused_launch<float, false, 4>(shape, variant, tiles, ntiles, boxes, st);
  }
}
