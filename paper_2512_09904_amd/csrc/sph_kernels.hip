// sph_kernels.hip -- gfx950 kernels of the WCSPH thermo-fluid hot path
// (arXiv 2512.09904, Section 2).  One advection step is the launch sequence
// clear -> pose -> fold -> scan1..3 -> scatter -> cellsort -> reorder -> build
// -> dt -> visc_heat -> n_ac x (half_a, momentum, continuity, half_b) -> end
// -> final.  Every kernel covers all slots of a launch table: block b of the
// grid belongs to the slot whose block range contains b, so one launch
// steps many independent solves (continuous batching) and a solve's result
// does not depend on which other slots share the launch.
//
// No MFMA: the sweeps are gathers over neighbour rows, bound by HBM and
// cache bandwidth.  Reductions are deterministic (fixed-order wave
// butterflies and block trees, Neumaier-compensated FP64 for the reports);
// the only atomics are integer counters of the cell sort and fault flags.
#include <math.h>

#include "sph_internal.h"

namespace sphk {

// ---------------------------------------------------------------------------
// precision policies: position anchors, interaction arithmetic, temperature
// ---------------------------------------------------------------------------
struct PMixed {
  typedef double Pos;
  typedef float Real;
  typedef double Temp;
  static constexpr bool kRel = true;   // density stored as rho - rho0
};
struct PF64 {
  typedef double Pos;
  typedef double Real;
  typedef double Temp;
  static constexpr bool kRel = true;
};
struct PF32 {
  typedef float Pos;
  typedef float Real;
  typedef float Temp;
  static constexpr bool kRel = false;  // absolute density in FP32
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_slot(const LaunchTab& L, int dom, int& lb) {
  const int blk = blockIdx.x;
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

// per-thread accumulators for up to NACC (= 2) bodies touched by one fluid
// particle; explicit register arrays, selected by branches (no indexing by a
// runtime value, so nothing goes to scratch)
template <int W>
struct BodyAcc {
  int id0, id1;
  double v0[W], v1[W];
  __device__ void init() {
    id0 = id1 = -1;
#pragma unroll
    for (int k = 0; k < W; ++k) v0[k] = v1[k] = 0.0;
  }
  // adds x[0..W) to body b; false when both accumulators hold other bodies
  __device__ __forceinline__ bool add(int b, const double (&x)[W]) {
    const bool s0 = id0 < 0 || id0 == b;
    id0 = s0 ? b : id0;
    const bool s1 = !s0 && (id1 < 0 || id1 == b);
    id1 = s1 ? b : id1;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      v0[k] += s0 ? x[k] : 0.0;
      v1[k] += s1 ? x[k] : 0.0;
    }
    return s0 || s1;
  }
};

// Deterministic block reduction of per-thread body accumulators: for each
// body and component, wave butterfly then the four waves in order.
template <int W>
// out is quantity-major: out[(b * W + k) * nblk + lb]
__device__ __forceinline__ void block_body_reduce(const BodyAcc<W> acc, int nbody, double* out, size_t nblk,
                                                  int lb, bool accumulate, double* lds /* [4][NB][W] */) {
  const int wv = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
  for (int b = 0; b < nbody; ++b) {
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const double x = (acc.id0 == b ? acc.v0[k] : 0.0) + (acc.id1 == b ? acc.v1[k] : 0.0);
      const double s = wave_sum(x);
      if (ln == 0) lds[(wv * NB + b) * W + k] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < nbody * W) {
    const int b = threadIdx.x / W, k = threadIdx.x % W;
    double s = lds[(0 * NB + b) * W + k];
    s += lds[(1 * NB + b) * W + k];
    s += lds[(2 * NB + b) * W + k];
    s += lds[(3 * NB + b) * W + k];
    double* o = out + (size_t)(b * W + k) * nblk + lb;
    if (accumulate) *o += s;
    else *o = s;
  }
}

// ---------------------------------------------------------------------------
// K: clear per-cell counters
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_clear(const SlotDesc* table, LaunchTab tab) {
  SLOT_PROLOGUE(DOM_CELL);
  const int c = lb * BLOCK + threadIdx.x;
  if (c < S.ncells) {
    S.cnt_f[c] = 0u;
    S.cnt_s[c] = 0u;
  }
}

// ---------------------------------------------------------------------------
// K: prescribed rigid rotation of the bodies at the step's time (Section 4:
// gears turn at fixed speed and temperature).  Angle omega*t from the FP64
// time; Rodrigues rotation about the unit axis.  Also bins the solid particle
// into its cell and stages its arrays for the gather.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_pose(const SlotDesc* table, LaunchTab tab) {
#pragma clang fp contract(off)
  typedef typename P::Pos Pos;
  typedef typename P::Real Real;
  SLOT_PROLOGUE(DOM_SOLID);
  const int w = lb * BLOCK + threadIdx.x;
  const int ns = S.ns;
  if (w >= ns) return;
  const int b = S.body[w];
  const double th = S.bom[b] * S.ctl->t;
  double sn, cs;
  sincos(th, &sn, &cs);
  const double* a = S.ba[b];
  const double* ctr = S.bc[b];
  double u[3], n[3], ru[3], rn[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    u[k] = S.x0[k * ns + w] - ctr[k];
    n[k] = S.n0[k * ns + w];
  }
  {
    const double axu[3] = {a[1] * u[2] - a[2] * u[1], a[2] * u[0] - a[0] * u[2], a[0] * u[1] - a[1] * u[0]};
    const double au = a[0] * u[0] + a[1] * u[1] + a[2] * u[2];
    const double axn[3] = {a[1] * n[2] - a[2] * n[1], a[2] * n[0] - a[0] * n[2], a[0] * n[1] - a[1] * n[0]};
    const double an = a[0] * n[0] + a[1] * n[1] + a[2] * n[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ru[k] = u[k] * cs + axu[k] * sn + a[k] * au * (1.0 - cs);
      rn[k] = n[k] * cs + axn[k] * sn + a[k] * an * (1.0 - cs);
    }
  }
  const double om = S.bom[b];
  const double wa[3] = {om * a[0], om * a[1], om * a[2]};
  const double vw[3] = {wa[1] * ru[2] - wa[2] * ru[1], wa[2] * ru[0] - wa[0] * ru[2], wa[0] * ru[1] - wa[1] * ru[0]};
  Pos* xw = (Pos*)S.xwb;
  Real* nw = (Real*)S.nwb;
  Real* vv = (Real*)S.vwb;
  Real* lv = (Real*)S.levb;
  Pos xp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    xp[k] = (Pos)(ctr[k] + ru[k]);
    xw[k * ns + w] = xp[k];
    nw[k * ns + w] = (Real)rn[k];
    vv[k * ns + w] = (Real)vw[k];
    lv[k * ns + w] = (Real)ru[k];
    S.x0b[k * ns + w] = S.x0[k * ns + w];
    S.n0b[k * ns + w] = S.n0[k * ns + w];
  }
  S.bodyb[w] = b;
  S.sidb[w] = S.sid[w];
  int c[3];
  if (!cell_coords<Pos>(S, xp[0], xp[1], xp[2], c)) raise_flag(S, F_DOMAIN);
  const uint32_t r = S.rank[cell_linear(S, c[0], c[1], c[2])];
  S.scell[w] = r;
  atomicAdd(&S.cnt_s[r], 1u);
}

// ---------------------------------------------------------------------------
// K: fold the FP32 drift into the FP64 anchor, stage the fluid arrays for the
// gather, bin into cells, and per-block max |v| for the time step.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_fold(const SlotDesc* table, LaunchTab tab) {
  typedef typename P::Pos Pos;
  typedef typename P::Real Real;
  typedef typename P::Temp Temp;
  __shared__ float red[BLOCK / WAVE];
  SLOT_PROLOGUE(DOM_FLUID);
  const int nf = S.nf;
  const int i = lb * BLOCK + threadIdx.x;
  float vm = 0.0f;
  if (i < nf) {
    Pos* xa = (Pos*)S.xa;
    Pos* xa2 = (Pos*)S.xa2;
    Real* dr = (Real*)S.drift;
    const Real* v = (const Real*)S.v;
    Real* v2 = (Real*)S.v2;
    Pos x[3];
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      x[k] = xa[k * nf + i] + (Pos)dr[k * nf + i];
      xa2[k * nf + i] = x[k];
      dr[k * nf + i] = (Real)0;
      const Real vk = v[k * nf + i];
      v2[k * nf + i] = vk;
      finite = finite && isfinite((double)x[k]) && isfinite((double)vk);
    }
    const Real rs = ((const Real*)S.rho)[i];
    const Temp T = ((const Temp*)S.T)[i];
    ((Real*)S.rho2)[i] = rs;
    ((Real*)S.drho2)[i] = ((const Real*)S.drho)[i];
    ((Temp*)S.T2)[i] = T;
    S.fid2[i] = S.fid[i];
    finite = finite && isfinite((double)rs) && isfinite((double)T);
    if (!finite) raise_flag(S, F_NONFINITE);
    const float v0 = (float)v[i], v1 = (float)v[nf + i], vz = (float)v[2 * nf + i];
    vm = sqrtf(v0 * v0 + v1 * v1 + vz * vz);
    int c[3];
    if (!cell_coords<Pos>(S, x[0], x[1], x[2], c)) raise_flag(S, F_DOMAIN);
    const uint32_t r = S.rank[cell_linear(S, c[0], c[1], c[2])];
    S.fcell[i] = r;
    atomicAdd(&S.cnt_f[r], 1u);
  }
  vm = wave_max(vm);
  if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = vm;
  __syncthreads();
  if (threadIdx.x == 0)
    S.vmax_part[lb] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// ---------------------------------------------------------------------------
// K: exclusive scan of per-cell counts (three phases: block sums, per-slot scan
// of the block sums, block-local scan plus offset).  Resets counts to serve as
// scatter cursors.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds, uint32_t& total) {
  const int wv = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    uint32_t y = __shfl_up(x, o, WAVE);
    if (ln >= o) x += y;
  }
  if (ln == WAVE - 1) lds[wv] = x;
  __syncthreads();
  uint32_t off = 0;
  for (int k = 0; k < wv; ++k) off += lds[k];
  total = lds[0] + lds[1] + lds[2] + lds[3];
  __syncthreads();
  return off + x - v;
}

__global__ __launch_bounds__(BLOCK) void k_scan1(const SlotDesc* table, LaunchTab tab) {
  __shared__ uint32_t red[2][BLOCK / WAVE];
  SLOT_PROLOGUE(DOM_CELL);
  const int c = lb * BLOCK + threadIdx.x;
  uint32_t a = 0, b = 0;
  if (c < S.ncells) {
    a = S.cnt_f[c];
    b = S.cnt_s[c];
  }
  a = wave_sum_u(a);
  b = wave_sum_u(b);
  if (threadIdx.x % WAVE == 0) {
    red[0][threadIdx.x / WAVE] = a;
    red[1][threadIdx.x / WAVE] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    S.bsum_f[lb] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    S.bsum_s[lb] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

__global__ __launch_bounds__(BLOCK) void k_scan2(const SlotDesc* table, LaunchTab tab) {
  __shared__ uint32_t lds[BLOCK / WAVE];
  SLOT_PROLOGUE(DOM_SLOT);
  (void)lb;
  const int n = S.nblk[DOM_CELL];
  const int ch = (n + BLOCK - 1) / BLOCK;
  const int b0 = threadIdx.x * ch;
  const int b1 = min(n, b0 + ch);
  for (int set = 0; set < 2; ++set) {
    uint32_t* bs = set ? S.bsum_s : S.bsum_f;
    uint32_t* st = set ? S.start_s : S.start_f;
    uint32_t s = 0;
    for (int k = b0; k < b1; ++k) s += bs[k];
    uint32_t total;
    uint32_t off = block_excl_scan(s, lds, total);
    for (int k = b0; k < b1; ++k) {
      uint32_t t = bs[k];
      bs[k] = off;
      off += t;
    }
    if (threadIdx.x == 0) st[S.ncells] = total;
    __syncthreads();
  }
}

__global__ __launch_bounds__(BLOCK) void k_scan3(const SlotDesc* table, LaunchTab tab) {
  __shared__ uint32_t lds[BLOCK / WAVE];
  SLOT_PROLOGUE(DOM_CELL);
  const int c = lb * BLOCK + threadIdx.x;
  const bool act = c < S.ncells;
  uint32_t a = act ? S.cnt_f[c] : 0u;
  uint32_t b = act ? S.cnt_s[c] : 0u;
  uint32_t ta, tb;
  const uint32_t pa = block_excl_scan(a, lds, ta);
  const uint32_t pb = block_excl_scan(b, lds, tb);
  if (act) {
    S.start_f[c] = S.bsum_f[lb] + pa;
    S.start_s[c] = S.bsum_s[lb] + pb;
    S.cnt_f[c] = 0u;
    S.cnt_s[c] = 0u;
  }
}

// ---------------------------------------------------------------------------
// K: counting-sort scatter; then each cell's run is ordered by original id,
// which makes the order the unique (Morton cell, id) order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_scatter(const SlotDesc* table, LaunchTab tab, int which) {
  SLOT_PROLOGUE(which ? DOM_SOLID : DOM_FLUID);
  const int n = which ? S.ns : S.nf;
  const int i = lb * BLOCK + threadIdx.x;
  if (i >= n) return;
  const uint32_t* cell = which ? S.scell : S.fcell;
  const uint32_t* start = which ? S.start_s : S.start_f;
  uint32_t* cnt = which ? S.cnt_s : S.cnt_f;
  uint32_t* perm = which ? S.sperm : S.fperm;
  const uint32_t r = cell[i];
  const uint32_t pos = start[r] + atomicAdd(&cnt[r], 1u);
  perm[pos] = (uint32_t)i;
}

__device__ __forceinline__ void sort_run(uint32_t* perm, uint32_t b, uint32_t e, const uint32_t* id) {
  for (uint32_t k = b + 1; k < e; ++k) {
    const uint32_t key = perm[k];
    const uint32_t kid = id[key];
    uint32_t m = k;
    while (m > b && id[perm[m - 1]] > kid) {
      perm[m] = perm[m - 1];
      --m;
    }
    perm[m] = key;
  }
}

__global__ __launch_bounds__(BLOCK) void k_cellsort(const SlotDesc* table, LaunchTab tab) {
  SLOT_PROLOGUE(DOM_CELL);
  const int c = lb * BLOCK + threadIdx.x;
  if (c >= S.ncells) return;
  sort_run(S.fperm, S.start_f[c], S.start_f[c + 1], S.fid);
  sort_run(S.sperm, S.start_s[c], S.start_s[c + 1], S.sid);
}

// ---------------------------------------------------------------------------
// K: gather the staged arrays into cell-sorted order
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_reorder(const SlotDesc* table, LaunchTab tab, int which) {
  typedef typename P::Pos Pos;
  typedef typename P::Real Real;
  typedef typename P::Temp Temp;
  SLOT_PROLOGUE(which ? DOM_SOLID : DOM_FLUID);
  const int k = lb * BLOCK + threadIdx.x;
  if (!which) {
    const int nf = S.nf;
    if (k >= nf) return;
    const uint32_t s = S.fperm[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ((Pos*)S.xa)[a * nf + k] = ((const Pos*)S.xa2)[a * nf + s];
      ((Real*)S.v)[a * nf + k] = ((const Real*)S.v2)[a * nf + s];
    }
    ((Real*)S.rho)[k] = ((const Real*)S.rho2)[s];
    ((Real*)S.drho)[k] = ((const Real*)S.drho2)[s];
    ((Temp*)S.T)[k] = ((const Temp*)S.T2)[s];
    S.fid[k] = S.fid2[s];
  } else {
    const int ns = S.ns;
    if (k >= ns) return;
    const uint32_t s = S.sperm[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      S.x0[a * ns + k] = S.x0b[a * ns + s];
      S.n0[a * ns + k] = S.n0b[a * ns + s];
      ((Pos*)S.xw)[a * ns + k] = ((const Pos*)S.xwb)[a * ns + s];
      ((Real*)S.nw)[a * ns + k] = ((const Real*)S.nwb)[a * ns + s];
      ((Real*)S.vw)[a * ns + k] = ((const Real*)S.vwb)[a * ns + s];
      ((Real*)S.lev)[a * ns + k] = ((const Real*)S.levb)[a * ns + s];
    }
    S.body[k] = S.bodyb[s];
    S.sid[k] = S.sidb[s];
  }
}

// ---------------------------------------------------------------------------
// K: neighbour rows (Section 2.8: neighbour lists and kernel quantities are
// refreshed once per advection step).  The cutoff test d^2 < (2h)^2 is FP64
// with d^2 = (dx dx + dy dy) + dz dz and no contraction.  Each hit stores the
// neighbour index (the pair geometry r_ij, F is written by the first sweep,
// whose stores are coalesced).  The kernel sum (self, fluid, solid) drives the
// density re-initialisation of Section 2.4 (eq. 14 with a free surface, eq. 15
// without), against the perfect-lattice sum S0.
//
// A wavefront holds 64 consecutive particles of the Morton order, i.e. a few
// neighbouring cells.  It walks the cells of its lanes' bounding box (plus one
// layer) once; inside a cell every lane sees the same candidate, so candidate
// positions are wave-uniform (scalar) loads, and each lane keeps the
// candidates of its own 27-cell stencil.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, WAVE));
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WAVE));
  return __builtin_amdgcn_readfirstlane(v);
}

template <class P>
__global__ __launch_bounds__(BLOCK) void k_build(const SlotDesc* table, LaunchTab tab) {
#pragma clang fp contract(off)
  typedef typename P::Pos Pos;
  typedef typename P::Real Real;
  SLOT_PROLOGUE(DOM_FLUID);
  const int i = lb * BLOCK + threadIdx.x;
  const int nf = S.nf, ns = S.ns;
  const bool act = i < nf;
  const int ii = act ? i : nf - 1;
  const Pos* xa = (const Pos*)S.xa;
  const Pos* xw = (const Pos*)S.xw;
  const Pos xi = xa[ii], yi = xa[nf + ii], zi = xa[2 * nf + ii];
  int c[3];
  cell_coords<Pos>(S, xi, yi, zi, c);
  int lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = max(wave_min_i(c[a]) - 1, 0);
    hi[a] = min(wave_max_i(c[a]) + 1, S.dims[a] - 1);
  }
  const int lane = i & (WAVE - 1);
  const int64_t slice = i >> 6;
  const int64_t basef = slice * (int64_t)S.kf * WAVE + lane;
  const int64_t bases = slice * (int64_t)S.ks * WAVE + lane;
  const double h = S.h, cut2 = S.cut2, kW = S.kW;
  const int kf = S.kf, ks = S.ks;
  int cf = 0, cs = 0;
  double sw = kW;  // W(0)
  for (int cz = lo[2]; cz <= hi[2]; ++cz) {
    for (int cy = lo[1]; cy <= hi[1]; ++cy) {
      for (int cx = lo[0]; cx <= hi[0]; ++cx) {
        const bool need = act && abs(cx - c[0]) <= 1 && abs(cy - c[1]) <= 1 && abs(cz - c[2]) <= 1;
        if (!__any(need)) continue;
        const uint32_t r = S.rank[cell_linear(S, cx, cy, cz)];
        const uint32_t j0 = S.start_f[r], j1 = S.start_f[r + 1];
        for (uint32_t j = j0; j < j1; ++j) {
          const Pos ddx = xi - xa[j], ddy = yi - xa[nf + j], ddz = zi - xa[2 * nf + j];
          const Pos s2 = ddx * ddx + ddy * ddy;
          const Pos d2 = s2 + ddz * ddz;
          if (need && (int)j != i && (double)d2 < cut2) {
            const double rr = sqrt((double)d2);
            const double q = rr / h;
            const double t = 1.0 - 0.5 * q;
            sw += kW * t * t * t * t * (1.0 + 2.0 * q);
            if (cf < kf) S.nj[basef + (int64_t)cf * WAVE] = j;
            ++cf;
          }
        }
        const uint32_t w0 = S.start_s[r], w1 = S.start_s[r + 1];
        for (uint32_t w = w0; w < w1; ++w) {
          const Pos ddx = xi - xw[w], ddy = yi - xw[ns + w], ddz = zi - xw[2 * ns + w];
          const Pos s2 = ddx * ddx + ddy * ddy;
          const Pos d2 = s2 + ddz * ddz;
          if (need && (double)d2 < cut2) {
            const double rr = sqrt((double)d2);
            const double q = rr / h;
            const double t = 1.0 - 0.5 * q;
            sw += kW * t * t * t * t * (1.0 + 2.0 * q);
            if (cs < ks) S.sj[bases + (int64_t)cs * WAVE] = w;
            ++cs;
          }
        }
      }
    }
  }
  if (!act) return;
  if (cf > kf || cs > ks) {
    raise_flag(S, F_CAPACITY);
    cf = min(cf, kf);
    cs = min(cs, ks);
  }
  S.nfc[i] = (uint32_t)cf;
  S.nsc[i] = (uint32_t)cs;
  S.sumW[i] = sw;
  // density re-initialisation
  Real* rho = (Real*)S.rho;
  const double dp3 = S.dp * S.dp * S.dp;
  const double rre = S.rho0 * (dp3 * sw) / S.S0;
  const double rcur = P::kRel ? S.rho0 + (double)rho[i] : (double)rho[i];
  const double rn = S.free_surface ? fmax(rcur, rre) : rre;
  rho[i] = P::kRel ? (Real)(rn - S.rho0) : (Real)rn;
}

// ---------------------------------------------------------------------------
// K: dual-criteria time step (Section 2.8, eq. 25).  |v|max covers the fluid
// and the bodies' tip speeds; n_ac is capped by shortening dt_ad.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_dt(const SlotDesc* table, LaunchTab tab) {
  __shared__ float red[BLOCK / WAVE];
  SLOT_PROLOGUE(DOM_SLOT);
  (void)lb;
  const int n = S.nblk[DOM_FLUID];
  float m = 0.0f;
  for (int k = threadIdx.x; k < n; k += BLOCK) m = fmaxf(m, S.vmax_part[k]);
  m = wave_max(m);
  if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double vm = (double)fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  for (int b = 0; b < S.nbody; ++b) vm = fmax(vm, S.btip[b]);
  SlotCtl* C = S.ctl;
  double tad, dt;
  int nac;
  if (S.fixed_dt_ad > 0.0) {
    tad = S.fixed_dt_ad;
    nac = S.fixed_nac > 0 ? S.fixed_nac : 1;
    dt = tad / (double)nac;
  } else {
    const double h = S.h;
    const double visc = h * h / S.nu;
    const double adv = vm > 0.0 ? h / vm : visc;
    tad = S.cfl_ad * (adv < visc ? adv : visc);
    const double tac = S.cfl_ac * h / (S.c0 + vm);
    double nn = ceil(tad / tac);
    if (nn < 1.0) nn = 1.0;
    if (nn > (double)S.nac_bound) {
      nn = (double)S.nac_bound;
      tad = nn * tac;
    }
    nac = (int)nn;
    dt = tad / nn;
  }
  C->dt_ad = tad;
  C->dt = dt;
  C->n_ac = nac;
}

// Frozen pair geometry of a row entry: r_ij = x_i - x_j from the FP64 anchors
// (rounded to the interaction type) and F = (dW/dr)/r = kF (1 - q/2)^3 from
// the FP64 distance, evaluated exactly as in the build's cutoff test.
template <class Pos, class Real>
__device__ __forceinline__ Real pair_geom(const SlotDesc& S, Pos xi, Pos yi, Pos zi, Pos xj, Pos yj, Pos zj,
                                          Real& rx, Real& ry, Real& rz) {
#pragma clang fp contract(off)
  const Pos ddx = xi - xj, ddy = yi - yj, ddz = zi - zj;
  const Pos s2 = ddx * ddx + ddy * ddy;
  const Pos d2 = s2 + ddz * ddz;
  const double q = sqrt((double)d2) / S.h;
  const double t = 1.0 - 0.5 * q;
  rx = (Real)ddx;
  ry = (Real)ddy;
  rz = (Real)ddz;
  return (Real)(S.kF * t * t * t);
}

// ---------------------------------------------------------------------------
// K: viscous acceleration (eq. 10 fluid-fluid, eq. 18 fluid-wall) and heat
// conduction rate (eq. 22), both frozen for the advection step.  As the first
// sweep over fresh rows it also writes each row entry's pair geometry.  Per-block
// partials: viscous force and torque on each body and its heat flow into the
// fluid.  Also clears this block's pressure-force accumulators.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_visc_heat(const SlotDesc* table, LaunchTab tab) {
  typedef typename P::Real Real;
  typedef typename P::Temp Temp;
  __shared__ double lds[4 * NB * 7];
  SLOT_PROLOGUE(DOM_FLUID);
  const int nf = S.nf, ns = S.ns;
  const int i = lb * BLOCK + threadIdx.x;
  const size_t nbf = (size_t)S.nblk[DOM_FLUID];
  if (threadIdx.x < NB * 6) S.press_part[(size_t)threadIdx.x * nbf + lb] = 0.0;
  BodyAcc<7> acc;
  acc.init();
  bool wall = false;
  if (i < nf) {
    const Real* v = (const Real*)S.v;
    const Real* rho = (const Real*)S.rho;
    const Temp* T = (const Temp*)S.T;
    const Real m = (Real)S.mass;
    const Real vix = v[i], viy = v[nf + i], viz = v[2 * nf + i];
    const Real rhoi = rho_abs<P>(S, rho[i]);
    const Temp Ti = T[i];
    const Real c2 = (Real)(2.0 * S.eta) * rcp(rhoi);   // 2 eta V_i / m_i
    const Real Kff = (Real)(4.0 * S.k_f * S.k_f / (S.k_f + S.k_f));
    Real ax = 0, ay = 0, az = 0, hs = 0;
    const int lane = i & (WAVE - 1);
    const int64_t slice = i >> 6;
    typedef typename P::Pos Pos;
    const Pos* xa = (const Pos*)S.xa;
    const Pos xi = xa[i], yi = xa[nf + i], zi = xa[2 * nf + i];
    {
      const int n = (int)S.nfc[i];
      const int64_t base = slice * (int64_t)S.kf * WAVE + lane;
      Real* R = (Real*)S.nr;
      Real* F = (Real*)S.nF;
      const int64_t L = S.rowlen_f;
      for (int k = 0; k < n; ++k) {
        const int64_t o = base + (int64_t)k * WAVE;
        const uint32_t j = S.nj[o];
        Real rx, ry, rz;
        const Real Fk = pair_geom<Pos, Real>(S, xi, yi, zi, xa[j], xa[nf + j], xa[2 * nf + j], rx, ry, rz);
        R[o] = rx;
        R[L + o] = ry;
        R[2 * L + o] = rz;
        F[o] = Fk;
        const Real Vj = m * rcp(rho_abs<P>(S, rho[j]));
        const Real cv = c2 * Vj * Fk;
        ax += cv * (vix - v[j]);
        ay += cv * (viy - v[nf + j]);
        az += cv * (viz - v[2 * nf + j]);
        hs += Vj * Kff * (Real)(Ti - T[j]) * Fk;
      }
    }
    {
      const int n = (int)S.nsc[i];
      wall = n > 0;
      const int64_t base = slice * (int64_t)S.ks * WAVE + lane;
      Real* R = (Real*)S.sr;
      Real* F = (Real*)S.sF;
      const int64_t L = S.rowlen_s;
      const Pos* xw = (const Pos*)S.xw;
      const Real* vw = (const Real*)S.vw;
      const Real* lv = (const Real*)S.lev;
      const Real Vw = (Real)S.vol_w;
      const Real rc = rcp(rhoi * (Real)S.cp_f);
      for (int k = 0; k < n; ++k) {
        const int64_t o = base + (int64_t)k * WAVE;
        const uint32_t w = S.sj[o];
        Real rx, ry, rz;
        const Real Fk = pair_geom<Pos, Real>(S, xi, yi, zi, xw[w], xw[ns + w], xw[2 * ns + w], rx, ry, rz);
        R[o] = rx;
        R[L + o] = ry;
        R[2 * L + o] = rz;
        F[o] = Fk;
        const int b = S.body[w];
        const Real cv = c2 * Vw * Fk;
        const Real fx = cv * (vix - vw[w]), fy = cv * (viy - vw[ns + w]), fz = cv * (viz - vw[2 * ns + w]);
        ax += fx;
        ay += fy;
        az += fz;
        const Real Kiw = (Real)(4.0 * S.k_f * S.bk[b] / (S.k_f + S.bk[b]));
        const Real term = Vw * Kiw * (Real)(Ti - (Temp)S.bT[b]) * Fk;
        hs += term;
        // force of the fluid on the body is -m_i times this pair's acceleration
        const double gx = -(double)m * fx, gy = -(double)m * fy, gz = -(double)m * fz;
        const double lx = lv[w], ly = lv[ns + w], lz = lv[2 * ns + w];
        const double contrib[7] = {gx, gy, gz, ly * gz - lz * gy, lz * gx - lx * gz, lx * gy - ly * gx,
                                   (double)m * (double)S.cp_f * (double)(rc * term)};
        if (!acc.add(b, contrib)) raise_flag(S, F_CAPACITY);
      }
      Real* av = (Real*)S.av;
      av[i] = ax;
      av[nf + i] = ay;
      av[2 * nf + i] = az;
      ((Real*)S.dTdt)[i] = rc * hs;
    }
  }
  if (__syncthreads_or(wall))
    block_body_reduce<7>(acc, S.nbody, S.visc_part, nbf, lb, false, lds);
  else if (threadIdx.x < NB * 7)
    S.visc_part[(size_t)threadIdx.x * nbf + lb] = 0.0;
}

// ---------------------------------------------------------------------------
// K: first half of an acoustic sub-step: rho += dt/2 Drho, x += dt/2 v
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_half_a(const SlotDesc* table, LaunchTab tab, int sub) {
  typedef typename P::Real Real;
  SLOT_PROLOGUE(DOM_FLUID);
  if (sub >= S.ctl->n_ac) return;
  const int nf = S.nf;
  const int i = lb * BLOCK + threadIdx.x;
  if (i >= nf) return;
  const Real hdt = (Real)(0.5 * S.ctl->dt);
  Real* rho = (Real*)S.rho;
  rho[i] += hdt * ((const Real*)S.drho)[i];
  Real* dr = (Real*)S.drift;
  const Real* v = (const Real*)S.v;
#pragma unroll
  for (int k = 0; k < 3; ++k) dr[k * nf + i] += hdt * v[k * nf + i];
}

// ---------------------------------------------------------------------------
// K: Riemann momentum (eq. 10-12) with the wall pressure of the one-sided
// problem (eq. 16-19); v_new = v + dt (a_p + a_visc + g), then the second
// half drift x += dt/2 v_new.  Per-block pressure force and torque on each
// body accumulate over the sub-steps.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_momentum(const SlotDesc* table, LaunchTab tab, int sub) {
  typedef typename P::Real Real;
  __shared__ double lds[4 * NB * 6];
  SLOT_PROLOGUE(DOM_FLUID);
  if (sub >= S.ctl->n_ac) return;
  const int nf = S.nf, ns = S.ns;
  const int i = lb * BLOCK + threadIdx.x;
  BodyAcc<6> acc;
  acc.init();
  bool wall = false;
  if (i < nf) {
    const Real* v = (const Real*)S.v;
    const Real* rho = (const Real*)S.rho;
    const Real c0 = (Real)S.c0;
    const Real m = (Real)S.mass;
    const Real vix = v[i], viy = v[nf + i], viz = v[2 * nf + i];
    const Real rs = rho[i];
    const Real rhoi = rho_abs<P>(S, rs);
    const Real pi = press<P>(S, rs);
    const Real c2 = (Real)2 * rcp(rhoi);   // 2 V_i / m_i
    Real ax = 0, ay = 0, az = 0;
    const int lane = i & (WAVE - 1);
    const int64_t slice = i >> 6;
    {
      const int n = (int)S.nfc[i];
      const int64_t base = slice * (int64_t)S.kf * WAVE + lane;
      const Real* R = (const Real*)S.nr;
      const Real* F = (const Real*)S.nF;
      const int64_t L = S.rowlen_f;
      for (int k = 0; k < n; ++k) {
        const int64_t o = base + (int64_t)k * WAVE;
        const uint32_t j = S.nj[o];
        const Real rx = R[o], ry = R[L + o], rz = R[2 * L + o], Fk = F[o];
        const Real r2 = rx * rx + ry * ry + rz * rz;
        if (r2 == (Real)0) continue;
        const Real inv = rsq(r2);
        const Real rsj = rho[j];
        const Real rhoj = rho_abs<P>(S, rsj);
        const Real pj = press<P>(S, rsj);
        // U_L - U_R = -(v_i - v_j) . e_ij
        const Real dU = -((vix - v[j]) * rx + (viy - v[nf + j]) * ry + (viz - v[2 * nf + j]) * rz) * inv;
        const Real beta = fmin((Real)3 * fmax(dU, (Real)0), c0);
        const Real ps = (Real)0.5 * (pi + pj) + rhoi * rhoj * beta * dU * rcp(rhoi + rhoj);
        const Real s = -c2 * (m * rcp(rhoj)) * ps * Fk;
        ax += s * rx;
        ay += s * ry;
        az += s * rz;
      }
    }
    {
      const int n = (int)S.nsc[i];
      wall = n > 0;
      const int64_t base = slice * (int64_t)S.ks * WAVE + lane;
      const Real* R = (const Real*)S.sr;
      const Real* F = (const Real*)S.sF;
      const Real* lv = (const Real*)S.lev;
      const int64_t L = S.rowlen_s;
      const Real gx = (Real)S.g[0], gy = (Real)S.g[1], gz = (Real)S.g[2];
      const Real rho0 = (Real)S.rho0;
      const Real ic02 = (Real)(1.0 / (S.c0 * S.c0));
      const Real Vw = (Real)S.vol_w;
      for (int k = 0; k < n; ++k) {
        const int64_t o = base + (int64_t)k * WAVE;
        const uint32_t w = S.sj[o];
        const Real rx = R[o], ry = R[L + o], rz = R[2 * L + o], Fk = F[o];
        // right state of eq. 17: P_R = P_L + rho_f g . (x_w - x_f), rho_R from the EoS
        const Real PR = pi - rhoi * (gx * rx + gy * ry + gz * rz);
        const Real rhoR = rho0 + PR * ic02;
        const Real ps = (rhoi * PR + rhoR * pi) * rcp(rhoi + rhoR);   // eq. 19
        const Real s = -c2 * Vw * ps * Fk;
        const Real fx = s * rx, fy = s * ry, fz = s * rz;
        ax += fx;
        ay += fy;
        az += fz;
        const double hx = -(double)m * fx, hy = -(double)m * fy, hz = -(double)m * fz;
        const double lx = lv[w], ly = lv[ns + w], lz = lv[2 * ns + w];
        const double contrib[6] = {hx, hy, hz, ly * hz - lz * hy, lz * hx - lx * hz, lx * hy - ly * hx};
        if (!acc.add(S.body[w], contrib)) raise_flag(S, F_CAPACITY);
      }
    }
    const Real dt = (Real)S.ctl->dt;
    const Real hdt = (Real)(0.5 * S.ctl->dt);
    const Real* av = (const Real*)S.av;
    Real* vn = (Real*)S.vnew;
    Real* dr = (Real*)S.drift;
    const Real nx = vix + dt * (ax + av[i] + (Real)S.g[0]);
    const Real ny = viy + dt * (ay + av[nf + i] + (Real)S.g[1]);
    const Real nz = viz + dt * (az + av[2 * nf + i] + (Real)S.g[2]);
    vn[i] = nx;
    vn[nf + i] = ny;
    vn[2 * nf + i] = nz;
    dr[i] += hdt * nx;
    dr[nf + i] += hdt * ny;
    dr[2 * nf + i] += hdt * nz;
  }
  if (__syncthreads_or(wall))
    block_body_reduce<6>(acc, S.nbody, S.press_part, (size_t)S.nblk[DOM_FLUID], lb, true, lds);
}

// ---------------------------------------------------------------------------
// K: Riemann continuity (eq. 10, 11-13) with (v_i - v*) . e_ij = U* - U_L, and
// the wall's mirror state; writes Drho and commits v <- v_new.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_continuity(const SlotDesc* table, LaunchTab tab, int sub) {
  typedef typename P::Real Real;
  SLOT_PROLOGUE(DOM_FLUID);
  if (sub >= S.ctl->n_ac) return;
  const int nf = S.nf, ns = S.ns;
  const int i = lb * BLOCK + threadIdx.x;
  if (i >= nf) return;
  const Real* v = (const Real*)S.vnew;
  const Real* rho = (const Real*)S.rho;
  const Real c0 = (Real)S.c0;
  const Real m = (Real)S.mass;
  const Real vix = v[i], viy = v[nf + i], viz = v[2 * nf + i];
  const Real rs = rho[i];
  const Real rhoi = rho_abs<P>(S, rs);
  const Real pi = press<P>(S, rs);
  Real sum = 0;
  const int lane = i & (WAVE - 1);
  const int64_t slice = i >> 6;
  {
    const int n = (int)S.nfc[i];
    const int64_t base = slice * (int64_t)S.kf * WAVE + lane;
    const Real* R = (const Real*)S.nr;
    const Real* F = (const Real*)S.nF;
    const int64_t L = S.rowlen_f;
    for (int k = 0; k < n; ++k) {
      const int64_t o = base + (int64_t)k * WAVE;
      const uint32_t j = S.nj[o];
      const Real rx = R[o], ry = R[L + o], rz = R[2 * L + o], Fk = F[o];
      const Real r2 = rx * rx + ry * ry + rz * rz;
      if (r2 == (Real)0) continue;
      const Real rr = r2 * rsq(r2);
      const Real rsj = rho[j];
      const Real rhoj = rho_abs<P>(S, rsj);
      const Real pj = press<P>(S, rsj);
      // (U* - U_L) dW = [ (v_i - v_j) . r / 2 + (p_i - p_j) r / (c0 (rho_i + rho_j)) ] F
      const Real vr = (vix - v[j]) * rx + (viy - v[nf + j]) * ry + (viz - v[2 * nf + j]) * rz;
      const Real dv = (Real)0.5 * vr + (pi - pj) * rr * rcp(c0 * (rhoi + rhoj));
      sum += (m * rcp(rhoj)) * dv * Fk;
    }
  }
  {
    const int n = (int)S.nsc[i];
    const int64_t base = slice * (int64_t)S.ks * WAVE + lane;
    const Real* R = (const Real*)S.sr;
    const Real* F = (const Real*)S.sF;
    const Real* nw = (const Real*)S.nw;
    const Real* vw = (const Real*)S.vw;
    const int64_t L = S.rowlen_s;
    const Real gx = (Real)S.g[0], gy = (Real)S.g[1], gz = (Real)S.g[2];
    const Real rho0 = (Real)S.rho0;
    const Real ic02 = (Real)(1.0 / (S.c0 * S.c0));
    const Real Vw = (Real)S.vol_w;
    for (int k = 0; k < n; ++k) {
      const int64_t o = base + (int64_t)k * WAVE;
      const uint32_t w = S.sj[o];
      const Real rx = R[o], ry = R[L + o], rz = R[2 * L + o], Fk = F[o];
      const Real nx = nw[w], ny = nw[ns + w], nz = nw[2 * ns + w];
      const Real PR = pi - rhoi * (gx * rx + gy * ry + gz * rz);
      const Real rhoR = rho0 + PR * ic02;
      const Real UL = -(nx * vix + ny * viy + nz * viz);
      const Real uw = -(nx * vw[w] + ny * vw[ns + w] + nz * vw[2 * ns + w]);
      const Real Us = uw + (pi - PR) * rcp(c0 * (rhoi + rhoR));
      sum += Vw * (Us - UL) * (nx * rx + ny * ry + nz * rz) * Fk;
    }
  }
  ((Real*)S.drho)[i] = (Real)2 * rhoi * sum;
  Real* vc = (Real*)S.v;
  vc[i] = vix;
  vc[nf + i] = viy;
  vc[2 * nf + i] = viz;
}

// ---------------------------------------------------------------------------
// K: second half of the density update: rho += dt/2 Drho
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_half_b(const SlotDesc* table, LaunchTab tab, int sub) {
  typedef typename P::Real Real;
  SLOT_PROLOGUE(DOM_FLUID);
  if (sub >= S.ctl->n_ac) return;
  const int i = lb * BLOCK + threadIdx.x;
  if (i >= S.nf) return;
  Real* rho = (Real*)S.rho;
  rho[i] += (Real)(0.5 * S.ctl->dt) * ((const Real*)S.drho)[i];
}

// ---------------------------------------------------------------------------
// K: temperature by explicit Euler over the advection step (eq. 22, 26), and
// per-block totals: mass, kinetic energy, thermal energy, sum rho dp^3, vmax.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_end(const SlotDesc* table, LaunchTab tab) {
  typedef typename P::Real Real;
  typedef typename P::Temp Temp;
  __shared__ double lds[BLOCK / WAVE][NGLOB];
  SLOT_PROLOGUE(DOM_FLUID);
  const int nf = S.nf;
  const int i = lb * BLOCK + threadIdx.x;
  double q[NGLOB] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < nf) {
    Temp* T = (Temp*)S.T;
    const Temp Tn = T[i] + (Temp)S.ctl->dt_ad * (Temp)((const Real*)S.dTdt)[i];
    T[i] = Tn;
    const Real* v = (const Real*)S.v;
    const double vx = v[i], vy = v[nf + i], vz = v[2 * nf + i];
    const double v2 = vx * vx + vy * vy + vz * vz;
    const double r = P::kRel ? S.rho0 + (double)((const Real*)S.rho)[i] : (double)((const Real*)S.rho)[i];
    q[0] = S.mass;
    q[1] = 0.5 * S.mass * v2;
    q[2] = S.mass * S.cp_f * (double)Tn;
    q[3] = r * (S.dp * S.dp * S.dp);
    q[4] = sqrt(v2);
    if (!isfinite(v2) || !isfinite(r) || !isfinite((double)Tn)) raise_flag(S, F_NONFINITE);
  }
  const int wv = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
#pragma unroll
  for (int k = 0; k < NGLOB - 1; ++k) {
    const double s = wave_sum(q[k]);
    if (ln == 0) lds[wv][k] = s;
  }
  {
    double md = q[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) md = fmax(md, __shfl_xor(md, o, WAVE));
    if (ln == 0) lds[wv][4] = md;
  }
  __syncthreads();
  if (threadIdx.x < NGLOB) {
    const int k = threadIdx.x;
    double s;
    if (k == 4) s = fmax(fmax(lds[0][4], lds[1][4]), fmax(lds[2][4], lds[3][4]));
    else s = ((lds[0][k] + lds[1][k]) + lds[2][k]) + lds[3][k];
    S.glob_part[(size_t)k * S.nblk[DOM_FLUID] + lb] = s;
  }
}

// ---------------------------------------------------------------------------
// K: per-slot reports: compensated sums of the block partials in fixed order,
// per-body force, torque, axial torque, power and heat flow; time integrals;
// advance t and the step counter.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_final(const SlotDesc* table, LaunchTab tab) {
  __shared__ double res[NGLOB + NB * 13];
  SLOT_PROLOGUE(DOM_SLOT);
  (void)lb;
  const int nblk = S.nblk[DOM_FLUID];
  const int nq = NGLOB + S.nbody * 13;
  const int wv = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
  for (int qi = wv; qi < nq; qi += BLOCK / WAVE) {
    // quantity qi: global k, or body b component c (7 viscous then 6 pressure)
    // partials are quantity-major: src[q * nblk + block]
    const double* src;
    bool is_max = false;
    if (qi < NGLOB) {
      src = S.glob_part + (size_t)qi * nblk;
      is_max = qi == 4;
    } else {
      const int b = (qi - NGLOB) / 13, c = (qi - NGLOB) % 13;
      src = c < 7 ? S.visc_part + (size_t)(b * 7 + c) * nblk : S.press_part + (size_t)(b * 6 + c - 7) * nblk;
    }
    if (is_max) {
      double m = 0.0;
      for (int k = ln; k < nblk; k += WAVE) m = fmax(m, src[k]);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, WAVE));
      if (ln == 0) res[qi] = m;
    } else {
      KS ks = {0.0, 0.0};
      for (int k = ln; k < nblk; k += WAVE) ks_add(ks, src[k]);
      ks = wave_ks(ks);
      if (ln == 0) res[qi] = ks.s + ks.c;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  SlotCtl* C = S.ctl;
  const double tad = C->dt_ad;
  const double inv_nac = 1.0 / (double)C->n_ac;
  double qsum = 0.0;
  bool finite = true;
  for (int b = 0; b < S.nbody; ++b) {
    const double* r = res + NGLOB + b * 13;
    sph_body_report& br = C->brep[b];
    for (int k = 0; k < 3; ++k) {
      br.force[k] = r[k] + r[7 + k] * inv_nac;
      br.torque[k] = r[3 + k] + r[10 + k] * inv_nac;
    }
    const double* a = S.ba[b];
    br.torque_axis = a[0] * br.torque[0] + a[1] * br.torque[1] + a[2] * br.torque[2];
    br.power = -S.bom[b] * br.torque_axis;
    br.heat_rate = r[6];
    C->cum[b][0] += tad * br.torque_axis;
    C->cum[b][1] += tad * br.power;
    C->cum[b][2] += tad * br.heat_rate;
    br.torque_axis_int = C->cum[b][0];
    br.energy_int = C->cum[b][1];
    br.heat_int = C->cum[b][2];
    qsum += br.heat_rate;
    finite = finite && isfinite(br.torque_axis) && isfinite(br.heat_rate) && isfinite(br.force[0]) &&
             isfinite(br.force[1]) && isfinite(br.force[2]);
  }
  C->t += tad;
  C->step += 1;
  C->substeps += C->n_ac;
  const double hs = tad * qsum;
  C->heat_total += hs;
  sph_report& R = C->rep;
  R.t = C->t;
  R.step = C->step;
  R.n_ac = C->n_ac;
  R.dt_ad = tad;
  R.dt = C->dt;
  R.mass = res[0];
  R.kinetic = res[1];
  R.thermal = res[2];
  R.mass_proxy = res[3];
  R.vmax = res[4];
  R.heat_step = hs;
  R.heat_total = C->heat_total;
  R.substeps = C->substeps;
  finite = finite && isfinite(res[1]) && isfinite(res[2]) && isfinite(res[3]);
  if (!finite) C->flags |= F_NONFINITE;
  R.flags = (int32_t)C->flags;
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
int grid_domain(int kid, int which) {
  switch (kid) {
    case SPH_K_CLEAR:
    case SPH_K_SCAN1:
    case SPH_K_SCAN3:
    case SPH_K_CELLSORT:
      return DOM_CELL;
    case SPH_K_POSE:
      return DOM_SOLID;
    case SPH_K_SCAN2:
    case SPH_K_DT:
    case SPH_K_FINAL:
      return DOM_SLOT;
    case SPH_K_SCATTER:
    case SPH_K_REORDER:
      return which ? DOM_SOLID : DOM_FLUID;
    default:
      return DOM_FLUID;
  }
}

template <class P>
static hipError_t launch_p(int kid, int which, int sub, const SlotDesc* T, const LaunchTab& L,
                           hipStream_t st) {
  const int dom = grid_domain(kid, which);
  const int nblk = L.blk0[dom][L.n];
  if (nblk <= 0) return hipSuccess;
  const dim3 g(nblk), b(BLOCK);
  switch (kid) {
    case SPH_K_CLEAR: hipLaunchKernelGGL(k_clear, g, b, 0, st, T, L); break;
    case SPH_K_POSE: hipLaunchKernelGGL(k_pose<P>, g, b, 0, st, T, L); break;
    case SPH_K_FOLD: hipLaunchKernelGGL(k_fold<P>, g, b, 0, st, T, L); break;
    case SPH_K_SCAN1: hipLaunchKernelGGL(k_scan1, g, b, 0, st, T, L); break;
    case SPH_K_SCAN2: hipLaunchKernelGGL(k_scan2, g, b, 0, st, T, L); break;
    case SPH_K_SCAN3: hipLaunchKernelGGL(k_scan3, g, b, 0, st, T, L); break;
    case SPH_K_SCATTER: hipLaunchKernelGGL(k_scatter, g, b, 0, st, T, L, which); break;
    case SPH_K_CELLSORT: hipLaunchKernelGGL(k_cellsort, g, b, 0, st, T, L); break;
    case SPH_K_REORDER: hipLaunchKernelGGL(k_reorder<P>, g, b, 0, st, T, L, which); break;
    case SPH_K_BUILD: hipLaunchKernelGGL(k_build<P>, g, b, 0, st, T, L); break;
    case SPH_K_DT: hipLaunchKernelGGL(k_dt, g, b, 0, st, T, L); break;
    case SPH_K_VISC_HEAT: hipLaunchKernelGGL(k_visc_heat<P>, g, b, 0, st, T, L); break;
    case SPH_K_HALF_A: hipLaunchKernelGGL(k_half_a<P>, g, b, 0, st, T, L, sub); break;
    case SPH_K_MOMENTUM: hipLaunchKernelGGL(k_momentum<P>, g, b, 0, st, T, L, sub); break;
    case SPH_K_CONTINUITY: hipLaunchKernelGGL(k_continuity<P>, g, b, 0, st, T, L, sub); break;
    case SPH_K_HALF_B: hipLaunchKernelGGL(k_half_b<P>, g, b, 0, st, T, L, sub); break;
    case SPH_K_END: hipLaunchKernelGGL(k_end<P>, g, b, 0, st, T, L); break;
    case SPH_K_FINAL: hipLaunchKernelGGL(k_final, g, b, 0, st, T, L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_kernel(int prec, int kid, int which, int sub, const SlotDesc* table,
                         const LaunchTab& tab, hipStream_t stream) {
  switch (prec) {
    case SPH_PREC_MIXED: return launch_p<PMixed>(kid, which, sub, table, tab, stream);
    case SPH_PREC_FP64: return launch_p<PF64>(kid, which, sub, table, tab, stream);
    case SPH_PREC_FP32: return launch_p<PF32>(kid, which, sub, table, tab, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sphk
