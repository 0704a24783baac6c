// Device helpers shared by the kernel translation units (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "sh_internal.h"

#pragma clang fp contract(off)


// ---------------------------------------------------------------------------------
// Per-stage scalars from the level's device scalars.  The right-hand side of stage s is
// evaluated at eta_n + c_s dt (c_s = stage_frac(s)); the EOM coefficients are
// c_fric = alpha/eta_s and c_pot = lambda * eta_s^beta.
// ---------------------------------------------------------------------------------
struct StageScal {
  double cf, cp, inv_dx2, h6, h3, h2, h1;
};

__device__ __forceinline__ double ipow(double x, int b) {
  double p = 1.0;
  for (int i = 0; i < b; ++i) p = p * x;
  return p;
}

__device__ __forceinline__ double level_time(const LevelScal& L) {
  return L.eta0 + (double)L.k * L.dt;
}

__device__ __forceinline__ StageScal stage_scalars(const LevelScal& L, int s) {
  const double eta_s = level_time(L) + stage_frac(s) * L.dt;
  StageScal r;
  r.cf = L.alpha / eta_s;
  r.cp = L.lam * ipow(eta_s, L.beta);
  r.inv_dx2 = L.inv_dx2;
  r.h6 = L.dt / 6.0;
  r.h3 = L.dt / 3.0;
  r.h2 = L.dt * 0.5;
  r.h1 = L.dt;
  return r;
}

// The stage scalars are the same for every lane; saying so keeps them in scalar
// registers instead of occupying vector registers for the whole kernel.
__device__ __forceinline__ double uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ StageScal uniform(const StageScal& s) {
  StageScal r;
  r.cf = uniform(s.cf);
  r.cp = uniform(s.cp);
  r.inv_dx2 = uniform(s.inv_dx2);
  r.h6 = uniform(s.h6);
  r.h3 = uniform(s.h3);
  r.h2 = uniform(s.h2);
  r.h1 = uniform(s.h1);
  return r;
}

// Base of a box's block in state slot `slot` (0..2).  Selecting with constant indices
// keeps the box record in registers (a computed index into it would go through memory).
__device__ __forceinline__ void* slot_base(const BoxDev& B, int slot) {
  return slot == 0 ? B.slot[0] : (slot == 1 ? B.slot[1] : B.slot[2]);
}

// Blocks are dispatched round-robin over the 8 XCDs of MI355X.  Map hardware block b
// to logical block (b % 8) * (n / 8) + b / 8 so that each XCD (with its own L2) works
// on one contiguous run of tiles, whose halo rows it then shares in its L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int nfull = n & ~7;
  if (b >= nfull) return b;
  return (b & 7) * (nfull >> 3) + (b >> 3);
}

// Element index of box-local cell (i, j, k), -ng <= i < nx + ng etc., in component 0.
template <typename T>
__device__ __forceinline__ long long elem(const BoxDev& B, int i, int j, int k) {
  return ((long long)(k + B.ng) * B.py + (j + B.ng)) * (long long)B.px + B.xoff + i;
}

// Box storage is global memory, but the box records hold generic pointers; reading it
// through pointers of the global address space lets the compiler use global (not flat)
// memory instructions.
template <typename T>
using Glob = __attribute__((address_space(1))) T;

// A level's scalars do not change while a kernel runs (only the counter kernel between
// launches writes them): read through the constant address space, a record at a
// wave-uniform address is fetched with scalar loads.
__device__ __forceinline__ LevelScal load_level(const LevelScal* p) {
  static_assert(sizeof(LevelScal) % 8 == 0, "whole 8-byte words");
  typedef const __attribute__((address_space(4))) unsigned long long* cq;
  unsigned long long w[sizeof(LevelScal) / 8];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(LevelScal) / 8); ++i) w[i] = ((cq)p)[i];
  LevelScal L;
  __builtin_memcpy(&L, w, sizeof(L));
  return L;
}

// Streams read or written once can be marked nontemporal so they do not displace data
// that neighbouring tiles re-read from L2.
template <bool NT, typename V>
__device__ __forceinline__ V ld(const V* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename V>
__device__ __forceinline__ V ld(const Glob<V>* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename P, typename V>
__device__ __forceinline__ void st(P p, V v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}


// Workgroup barrier that orders LDS accesses only.  __syncthreads() also waits for every
// outstanding global load of the wave, which would drain the plane prefetch of the
// z-marching kernels at each barrier; these exchange data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
