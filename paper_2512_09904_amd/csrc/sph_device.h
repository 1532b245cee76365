// sph_device.h -- device-side building blocks shared by the solver kernels
// (sph_kernels.hip) and the particle relaxation (sph_relax.hip): precision
// policies, slot lookup of a batched launch, wave reductions, cell and pair
// geometry of the frozen neighbour rows, and the Wendland C2 kernel factor.
#pragma once
#include <math.h>

#include <type_traits>

#include "sph_internal.h"

namespace sphk {

// ---------------------------------------------------------------------------
// precision policies: position anchors, interaction arithmetic, temperature
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

struct PMixed {
  typedef double Pos;
  typedef float Real;
  typedef double Temp;
  typedef d4 Pos4;
  typedef f4 Real4;
  static constexpr bool kRel = true;   // density stored as rho - rho0
};
struct PF64 {
  typedef double Pos;
  typedef double Real;
  typedef double Temp;
  typedef d4 Pos4;
  typedef d4 Real4;
  static constexpr bool kRel = true;
};
struct PF32 {
  typedef float Pos;
  typedef float Real;
  typedef float Temp;
  typedef f4 Pos4;
  typedef f4 Real4;
  static constexpr bool kRel = false;  // absolute density in FP32
};

// Arrays live in device global memory; loads through these pointers compile
// to global (not flat) memory instructions.
#define GLB __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLB T* gp(void* p) {
  return (GLB T*)p;
}
template <class T>
__device__ __forceinline__ const GLB T* gpc(const void* p) {
  return (const GLB T*)p;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Logical block numbers are laid out so that every XCD runs one
// contiguous range of blocks, i.e. one contiguous range of Morton-sorted
// particles, and the neighbour gathers of adjacent blocks hit the same L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_block(int b, int g) {
  const int q = g / NXCD, r = g % NXCD;
  const int x = b % NXCD, k = b / NXCD;
  return x * q + min(x, r) + k;
}

__device__ __forceinline__ int find_slot(const LaunchTab& L, int dom, int& lb) {
  const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
  int k = 0;
  for (int s = 1; s < L.n; ++s)
    if (blk >= L.blk0[dom][s]) k = s;
  lb = blk - L.blk0[dom][k];
  return L.slot[k];
}

__device__ __forceinline__ bool live(const SlotDesc& S) {
  return S.ctl->flags == 0u && S.ctl->step < S.ctl->target;
}

#define SLOT_PROLOGUE(DOM)                          \
  int lb_;                                          \
  const SlotDesc& S = table[find_slot(tab, DOM, lb_)]; \
  if (!live(S)) return;                             \
  const int lb = lb_;

__device__ __forceinline__ void raise_flag(const SlotDesc& S, uint32_t f) {
  atomicOr(&S.ctl->flags, f);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
  return v;
}
__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Neumaier-compensated accumulator (additions only, so no contraction applies)
struct KS {
  double s, c;
};
__device__ __forceinline__ void ks_add(KS& k, double x) {
  double t = k.s + x;
  if (fabs(k.s) >= fabs(x)) k.c += (k.s - t) + x;
  else k.c += (x - t) + k.s;
  k.s = t;
}
__device__ __forceinline__ KS wave_ks(KS k) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double s = __shfl_xor(k.s, o, WAVE);
    double c = __shfl_xor(k.c, o, WAVE);
    ks_add(k, s);
    k.c += c;
  }
  return k;
}

// cell of a point: floor((x - lo)/cs) per axis, FP64, correctly rounded
// division, no contraction.  Out-of-grid points are clamped and reported.
template <class PosT>
__device__ __forceinline__ bool cell_coords(const SlotDesc& S, PosT x, PosT y, PosT z, int c[3]) {
#pragma clang fp contract(off)
  const double p[3] = {(double)x, (double)y, (double)z};
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double f = floor((p[a] - S.lo[a]) / S.cs);
    if (!(f >= 0.0) || f >= (double)S.dims[a]) {
      ok = false;
      f = 0.0;
    }
    c[a] = (int)f;
  }
  return ok;
}

__device__ __forceinline__ int cell_linear(const SlotDesc& S, int cx, int cy, int cz) {
  return (cz * S.dims[1] + cy) * S.dims[0] + cx;
}

template <class P>
__device__ __forceinline__ typename P::Real rho_abs(const SlotDesc& S, typename P::Real s) {
  typedef typename P::Real Real;
  return P::kRel ? (Real)S.rho0 + s : s;
}
template <class P>
__device__ __forceinline__ typename P::Real press(const SlotDesc& S, typename P::Real s) {
  typedef typename P::Real Real;
  const Real c2 = (Real)(S.c0 * S.c0);
  return P::kRel ? c2 * s : c2 * (s - (Real)S.rho0);
}

// Reciprocal and reciprocal square root of the interaction type: the FP32
// hardware instructions (about 1 ulp) in the FP32 sweeps, IEEE operations in
// FP64 mode.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

// A 32-bit integer in the fourth lane of a 4-wide record: its bit pattern in
// FP32 (never a NaN: values stay below 2^30), its exact value in FP64.
__device__ __forceinline__ float pack_index(uint32_t j, float) { return __builtin_bit_cast(float, j); }
__device__ __forceinline__ double pack_index(uint32_t j, double) { return (double)j; }
__device__ __forceinline__ uint32_t unpack_index(float w) { return __builtin_bit_cast(uint32_t, w); }
__device__ __forceinline__ uint32_t unpack_index(double w) { return (uint32_t)w; }

// Cell-relative positions.  At the build every particle stores
// o = x - (lo + c cs_r) rounded to the interaction type, with its cell c
// packed as 10 bits per axis.  A pair's vector is then
//   r_ij = (o_i - o_j) + (c_i - c_j) cs_r,
// where c_i - c_j is -1, 0 or 1 per axis, so the second term is exact and
// r_ij carries only the offsets' roundings (a few ulp of cs_r), however far
// the particles are from the grid origin.
__device__ __forceinline__ uint32_t pack_cell(const int c[3]) {
  return (uint32_t)c[0] | (uint32_t)c[1] << 10 | (uint32_t)c[2] << 20;
}
template <class Real, class Real4>
__device__ __forceinline__ void pair_vec(const Real4 a, uint32_t ca, const Real4 b, Real csr, Real& rx, Real& ry,
                                         Real& rz) {
  const uint32_t cb = unpack_index(b.w);
  const int dx = (int)(ca & 1023u) - (int)(cb & 1023u);
  const int dy = (int)((ca >> 10) & 1023u) - (int)((cb >> 10) & 1023u);
  const int dz = (int)(ca >> 20) - (int)(cb >> 20);
  rx = (a.x - b.x) + (Real)dx * csr;
  ry = (a.y - b.y) + (Real)dy * csr;
  rz = (a.z - b.z) + (Real)dz * csr;
}
template <class P, class Pos>
__device__ __forceinline__ typename P::Real4 cell_offset(const SlotDesc& S, Pos x, Pos y, Pos z, const int c[3]) {
#pragma clang fp contract(off)
  typedef typename P::Real Real;
  typename P::Real4 o;
  o.x = (Real)((double)x - (S.lo[0] + (double)c[0] * S.cs_r));
  o.y = (Real)((double)y - (S.lo[1] + (double)c[1] * S.cs_r));
  o.z = (Real)((double)z - (S.lo[2] + (double)c[2] * S.cs_r));
  o.w = pack_index(pack_cell(c), (Real)0);
  return o;
}

// F = (dW/dr)/r = kF (1 - q/2)^3 of the Wendland C2 kernel from |r|^2
template <class Real>
__device__ __forceinline__ Real kernel_F(Real r2, Real inv_h, Real kF) {
  const Real q = r2 * rsq(r2) * inv_h;
  const Real t = (Real)1 - (Real)0.5 * q;
  return r2 > (Real)0 ? kF * t * t * t : kF;
}

// rows are streamed once per sweep: non-temporal loads keep them from
// evicting the gathered particle state in L2
template <class T>
__device__ __forceinline__ T ldnt(const GLB T* p) {
  return __builtin_nontemporal_load(p);
}

// block size of the single-block-per-slot kernels (reports, relaxation step)
constexpr int FINAL_BLOCK = 1024;

}  // namespace sphk
