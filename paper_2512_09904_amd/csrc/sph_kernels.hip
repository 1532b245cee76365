// sph_kernels.hip -- gfx950 kernels of the WCSPH thermo-fluid hot path
// (arXiv 2512.09904, Section 2).  One advection step is the launch sequence
// clear -> pose -> fold -> scan1..3 -> scatter -> cellsort -> reorder -> build
// -> sumw -> dt -> visc_heat -> half_a -> n_ac x (momentum, continuity) -> end
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

#include <type_traits>

#include "sph_device.h"

namespace sphk {

// Rows are walked ROW_UNROLL entries at a time (SOLID_UNROLL for the wall
// rows, VISC_SOLID_UNROLL for the viscous/heat sweep's wall rows, CONT_UNROLL
// in the continuity sweep, which runs fastest with twelve gathers in flight
// at three waves per SIMD: group sizes measured per sweep), and the next
// group's indices are loaded before the current group's gathers are
// consumed, so a wavefront keeps two dependent loads in flight.  Entries past
// a row's count are loaded from within the row's capacity (capacities are
// multiples of sixteen, a group beyond the first is loaded only when it
// starts below the count, and the continuity sweep's groups of twelve clamp
// their last loads to the row's last entry) and replaced by a null entry: own
// index, F = 0, which adds exactly zero to every sum.
#define ROW_UNROLL 8
#define SOLID_UNROLL 8
#define VISC_SOLID_UNROLL 4
#define CONT_UNROLL 12

// A block's window of the fluid anchors: the WIN particles around the
// block's own BLOCK (clamped to the array), staged in LDS with coalesced
// loads.  In the Morton order most neighbours of the block's particles fall
// inside it, so their 32-byte gathers become LDS reads; the rest are gathered
// from global memory.  Used by the FP64 kernel-sum sweep, whose anchor
// gathers (two 16-byte requests per pair) otherwise bound it by the vector
// memory unit's rate of one scattered lane per clock.  512 particles (16 KB
// of LDS per block) rather than 1024: fewer neighbours fall inside, but twice
// as many blocks fit on a CU, which the sweep gains more from beside the
// dummy-velocity sweep on the other stream.
constexpr int WIN = 512;
struct Window {
  uint32_t w0, wn;
};
__device__ __forceinline__ Window window_of(int lb, int nf) {
  Window w;
  w.wn = (uint32_t)min(WIN, nf);
  const int lo = lb * BLOCK - (WIN - BLOCK) / 2;
  w.w0 = (uint32_t)max(0, min(lo, nf - (int)w.wn));
  return w;
}
template <class T>
__device__ __forceinline__ void stage_window(T* lds, const GLB T* g, const Window& w) {
  for (uint32_t q = threadIdx.x; q < w.wn; q += BLOCK) lds[q] = g[w.w0 + q];
}
template <class T>
__device__ __forceinline__ T win_get(const T* lds, const GLB T* g, uint32_t j, const Window& w) {
  const uint32_t d = j - w.w0;
  return d < w.wn ? lds[d] : g[j];
}

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

// Counter increments of a wavefront whose lanes mostly share counters in
// runs (particles in last step's cell order): each run of consecutive active
// lanes with the same counter index does one atomic add of its length, and
// its lanes take consecutive values.  Inactive lanes form the wave's tail.
// Returns this lane's value of the counter before its own increment.
__device__ __forceinline__ uint32_t run_atomic_inc(uint32_t* cnt, uint32_t r, bool act) {
  const int lane = threadIdx.x & (WAVE - 1);
  const uint32_t prev = (uint32_t)__shfl_up((int)r, 1, WAVE);
  const uint64_t heads = __ballot(act && (lane == 0 || prev != r));
  const int nact = __popcll(__ballot(act));
  const uint64_t below = lane == WAVE - 1 ? ~0ull : ((2ull << lane) - 1);
  const uint64_t upto = heads & below;
  const int h = upto ? 63 - __builtin_clzll(upto) : 0;
  const uint64_t above = heads & ~below;
  const int next = above ? __builtin_ctzll(above) : nact;
  uint32_t old = 0;
  if (act && h == lane) old = atomicAdd(&cnt[r], (uint32_t)(next - lane));
  old = (uint32_t)__shfl((int)old, h, WAVE);
  return old + (uint32_t)(lane - h);
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
  typedef typename P::Pos4 Pos4;
  typedef typename P::Real4 Real4;
  SLOT_PROLOGUE(DOM_SOLID);
  const int w = lb * BLOCK + threadIdx.x;
  const bool act = w < S.ns;
  uint32_t r = 0;
  if (act) {
  const int b = S.body[w];
  const double th = S.bom[b] * S.ctl->t;
  double sn, cs;
  sincos(th, &sn, &cs);
  const double* a = S.ba[b];
  const double* ctr = S.bc[b];
  const d4 x0 = gpc<d4>(S.x0)[w];
  const d4 n0 = gpc<d4>(S.n0)[w];
  const double u[3] = {x0.x - ctr[0], x0.y - ctr[1], x0.z - ctr[2]};
  const double n[3] = {n0.x, n0.y, n0.z};
  double ru[3], rn[3];
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
  Pos4 xp;
  xp.x = (Pos)(ctr[0] + ru[0]);
  xp.y = (Pos)(ctr[1] + ru[1]);
  xp.z = (Pos)(ctr[2] + ru[2]);
  xp.w = (Pos)0;
  Real4 nw, vv, lv;
  nw.x = (Real)rn[0]; nw.y = (Real)rn[1]; nw.z = (Real)rn[2]; nw.w = (Real)0;
  vv.x = (Real)vw[0]; vv.y = (Real)vw[1]; vv.z = (Real)vw[2]; vv.w = (Real)0;
  lv.x = (Real)ru[0]; lv.y = (Real)ru[1]; lv.z = (Real)ru[2]; lv.w = (Real)b;
  gp<Pos4>(S.xwb)[w] = xp;
  gp<Real4>(S.nwb)[w] = nw;
  gp<Real4>(S.vwb)[w] = vv;
  gp<Real4>(S.levb)[w] = lv;
  gp<d4>(S.x0b)[w] = x0;
  gp<d4>(S.n0b)[w] = n0;
  S.bodyb[w] = b;
  S.sidb[w] = S.sid[w];
  int c[3];
  if (!cell_coords<Pos>(S, xp.x, xp.y, xp.z, c)) raise_flag(S, F_DOMAIN);
  r = S.rank[cell_linear(S, c[0], c[1], c[2])];
  S.scell[w] = r;
  }
  run_atomic_inc(S.cnt_s, r, act);
}

// ---------------------------------------------------------------------------
// K: fold the drift into the FP64 anchor, stage the fluid arrays for the
// gather, bin into cells, and per-block max |v| for the time step.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_fold(const SlotDesc* table, LaunchTab tab) {
  typedef typename P::Pos Pos;
  typedef typename P::Real Real;
  typedef typename P::Temp Temp;
  typedef typename P::Pos4 Pos4;
  typedef typename P::Real4 Real4;
  __shared__ double red[BLOCK / WAVE];
  SLOT_PROLOGUE(DOM_FLUID);
  const int i = lb * BLOCK + threadIdx.x;
  double vm = 0.0;
  uint32_t r = 0;
  if (i < S.nf) {
    Pos4 x = gpc<Pos4>(S.xa)[i];
    const Real4 d = gpc<Real4>(S.drift)[i];
    x.x += (Pos)d.x;
    x.y += (Pos)d.y;
    x.z += (Pos)d.z;
    gp<Pos4>(S.xa2)[i] = x;
    gp<Real4>(S.drift)[i] = Real4(0);
    const Real4 v = gpc<Real4>(S.vr)[i];
    gp<Real4>(S.vr2)[i] = v;
    gp<Real>(S.drho2)[i] = gpc<Real>(S.drho)[i];
    const Temp T = gpc<Temp>(S.T)[i];
    gp<Temp>(S.T2)[i] = T;
    S.fid2[i] = S.fid[i];
    if (S.mat) S.mat2[i] = S.mat[i];
    const bool finite = isfinite((double)x.x) && isfinite((double)x.y) && isfinite((double)x.z) &&
                        isfinite((double)v.x) && isfinite((double)v.y) && isfinite((double)v.z) &&
                        isfinite((double)v.w) && isfinite((double)T);
    if (!finite) raise_flag(S, F_NONFINITE);
    // |v| in FP64 from the stored components (eq. 25 takes the max)
    const double v0 = (double)v.x, v1 = (double)v.y, v2 = (double)v.z;
    vm = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    int c[3];
    if (!cell_coords<Pos>(S, x.x, x.y, x.z, c)) raise_flag(S, F_DOMAIN);
    r = S.rank[cell_linear(S, c[0], c[1], c[2])];
    S.fcell[i] = r;
  }
  run_atomic_inc(S.cnt_f, r, i < S.nf);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) vm = fmax(vm, __shfl_xor(vm, o, WAVE));
  if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = vm;
  __syncthreads();
  if (threadIdx.x == 0)
    S.vmax_part[lb] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
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
  const bool act = i < n;
  const uint32_t* cell = which ? S.scell : S.fcell;
  const uint32_t* start = which ? S.start_s : S.start_f;
  const uint32_t* id = which ? S.sidb : S.fid2;
  uint32_t* cnt = which ? S.cnt_s : S.cnt_f;
  uint64_t* key = which ? S.skey : S.fkey;
  const uint32_t r = act ? cell[i] : 0u;
  const uint32_t k = run_atomic_inc(cnt, r, act);
  if (act) key[start[r] + k] = (uint64_t)id[i] << 32 | (uint32_t)i;
}

// Orders each cell's run of keys (original id << 32 | staged index) by id and
// writes the staged indices in that order.  One thread per key position: the
// key's cell comes from its staged index, its rank in the cell is the number
// of the cell's keys below it (ids are unique, so the ranks are a
// permutation of the run), and its staged index goes to that place.  The
// lanes of a wavefront mostly share a cell, so the run's keys are read once
// per wavefront from cache, and the stores of a cell's permutation are
// contiguous.
__global__ __launch_bounds__(BLOCK) void k_cellsort(const SlotDesc* table, LaunchTab tab, int which) {
  SLOT_PROLOGUE(which ? DOM_SOLID : DOM_FLUID);
  const int n = which ? S.ns : S.nf;
  const int p = lb * BLOCK + threadIdx.x;
  if (p >= n) return;
  const uint64_t* key = which ? S.skey : S.fkey;
  const uint32_t* cell = which ? S.scell : S.fcell;
  const uint32_t* start = which ? S.start_s : S.start_f;
  uint32_t* perm = which ? S.sperm : S.fperm;
  const uint64_t kp = key[p];
  const uint32_t r = cell[(uint32_t)kp];
  const uint32_t b = start[r], e = start[r + 1];
  uint32_t rank = 0;
  for (uint32_t q = b; q < e; ++q) rank += key[q] < kp ? 1u : 0u;
  perm[b + rank] = (uint32_t)kp;
}

// A fluid particle's temperature and density rate side by side (16 bytes),
// so the fused first sub-step takes both of a neighbour's in one gather.
template <class P>
struct alignas(16) TempRate {
  typename P::Temp T;
  typename P::Real d;
};

// ---------------------------------------------------------------------------
// K: gather the staged arrays into cell-sorted order (fluid: also the
// (T, Drho) records)
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_reorder(const SlotDesc* table, LaunchTab tab, int which) {
  typedef typename P::Real Real;
  typedef typename P::Temp Temp;
  typedef typename P::Pos4 Pos4;
  typedef typename P::Real4 Real4;
  SLOT_PROLOGUE(which ? DOM_SOLID : DOM_FLUID);
  const int k = lb * BLOCK + threadIdx.x;
  if (!which) {
    if (k >= S.nf) return;
    const uint32_t s = S.fperm[k];
    gp<Pos4>(S.xa)[k] = gpc<Pos4>(S.xa2)[s];
    gp<Real4>(S.vr)[k] = gpc<Real4>(S.vr2)[s];
    const Real dr = gpc<Real>(S.drho2)[s];
    const Temp tk = gpc<Temp>(S.T2)[s];
    gp<Real>(S.drho)[k] = dr;
    gp<Temp>(S.T)[k] = tk;
    GLB TempRate<P>* td = gp<TempRate<P>>(S.td) + k;
    td->T = tk;
    td->d = dr;
    S.fid[k] = S.fid2[s];
    if (S.mat) S.mat[k] = S.mat2[s];
  } else {
    if (k >= S.ns) return;
    const uint32_t s = S.sperm[k];
    gp<d4>(S.x0)[k] = gpc<d4>(S.x0b)[s];
    gp<d4>(S.n0)[k] = gpc<d4>(S.n0b)[s];
    const Pos4 xp = gpc<Pos4>(S.xwb)[s];
    gp<Pos4>(S.xw)[k] = xp;
    int c[3];
    cell_coords<typename P::Pos>(S, xp.x, xp.y, xp.z, c);   // in the grid: checked by the pose
    gp<Real4>(S.so)[k] = cell_offset<P>(S, xp.x, xp.y, xp.z, c);
    gp<Real4>(S.nw)[k] = gpc<Real4>(S.nwb)[s];
    gp<Real4>(S.vw)[k] = gpc<Real4>(S.vwb)[s];
    gp<Real4>(S.lev)[k] = gpc<Real4>(S.levb)[s];
    S.body[k] = S.bodyb[s];
    S.sid[k] = S.sidb[s];
  }
}

// ---------------------------------------------------------------------------
// K: neighbour rows (Section 2.8: neighbour lists and kernel quantities are
// refreshed once per advection step).  The cutoff test d^2 < (2h)^2 is FP64
// with d^2 = (dx dx + dy dy) + dz dz and no contraction.  Every particle also
// stores its cell-relative position, from which the sweeps form r_ij.
//
// A wavefront holds 64 consecutive particles of the Morton order, i.e. runs
// of particles sharing a cell.  For each run the candidates of its 27-cell
// stencil are spread over the lanes in chunks of CB per lane, each candidate
// loaded once; for each chunk the run's particles are taken one at a time:
// each lane tests its candidates against the particle's position (broadcast
// from its lane into scalar registers), one ballot per candidate slot gives
// the hits, and the hit lanes write their indices to consecutive entries of
// the particle's row (particle-major, so a ballot's stores are contiguous;
// chunks of one run append in candidate order).  Every test is one
// of the particle's own stencil, and no lane waits on another's hits.  A row
// lists the stencil's cells in a fixed order, indices ascending within a
// cell.  At the end each lane moves its particle's row (still in cache) into
// the SELL layout the sweeps read, with stores contiguous across the wave.
// ---------------------------------------------------------------------------
// Wendland C2 weight W = kW (1 - q/2)^4 (1 + 2q), q = |r|/h, from d^2 in FP64.
// |r| comes from the hardware reciprocal square root refined by coupled
// Newton steps for sqrt(x) and 1/(2 sqrt(x)) (Goldschmidt's iteration) and a
// final residual correction, which leaves an error of about one ulp.
__device__ __forceinline__ double kernel_W_d2(double d2, double inv_h, double kW) {
  const double x = d2 > 0.0 ? d2 : 1.0;
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, hh = 0.5 * y;
  const double e = fma(-hh, g, 0.5);
  g = fma(g, e, g);
  hh = fma(hh, e, hh);
  const double res = fma(-g, g, x);
  g = fma(res, hh, g);
  const double q = (d2 > 0.0 ? g : 0.0) * inv_h;
  const double t = 1.0 - 0.5 * q;
  return kW * t * t * t * t * (1.0 + 2.0 * q);
}

// value of lane l (wave-uniform l) as a scalar
__device__ __forceinline__ float rl(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double rl(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Exclusive prefix sum over the wavefront's lanes; *total receives the sum.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total) {
  const int lane = threadIdx.x & (WAVE - 1);
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, d, WAVE);
    if (lane >= d) x += y;
  }
  *total = (uint32_t)__builtin_amdgcn_readlane((int)x, WAVE - 1);
  return x - v;
}

// LDS written by some lanes of a wavefront, then read by others
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Candidates of one run's stencil against the run's particles [L, R) of the
// wave.  pre/beg: per stencil cell (27) the prefix of candidate counts and the
// first index.  Hits of particle p go to row[p] + off, counted in lane p's cnt.
// candidate slots per lane: four keeps the build at five waves per SIMD
// (92 registers); eight (124 registers, four waves) was 3 % slower
constexpr int CB = 4;
template <class Pos, class Pos4>
__device__ __forceinline__ void run_candidates(const GLB Pos4* x, const uint32_t* pre, const uint32_t* beg,
                                               uint32_t M, int L, int R, int wbase, Pos xi, Pos yi, Pos zi,
                                               double cut2, GLB uint32_t* rows, int kr, int off, int cap,
                                               int& cnt, bool self) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & (WAVE - 1);
  for (uint32_t b0 = 0; b0 < M; b0 += (uint32_t)(WAVE * CB)) {
    Pos cx[CB], cy[CB], cz[CB];
    uint32_t cj[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      const uint32_t m = b0 + (uint32_t)(u * WAVE + lane);
      cj[u] = 0xffffffffu;
      cx[u] = cy[u] = cz[u] = (Pos)1e30;   // far: never a hit
      if (m < M) {
        int q = 0;
#pragma unroll
        for (int st = 16; st > 0; st >>= 1)
          if (q + st < 27 && pre[q + st] <= m) q += st;
        const uint32_t j = beg[q] + (m - pre[q]);
        const Pos4 pj = x[j];
        cj[u] = j;
        cx[u] = pj.x;
        cy[u] = pj.y;
        cz[u] = pj.z;
      }
    }
    const int nu = (int)min((uint32_t)CB, (M - b0 + WAVE - 1) / WAVE);
    for (int p = L; p < R; ++p) {
      const Pos px = rl(xi, p), py = rl(yi, p), pz = rl(zi, p);
      const uint32_t ip = (uint32_t)(wbase + p);
      int c = __builtin_amdgcn_readlane(cnt, p);
      GLB uint32_t* row = rows + (int64_t)ip * kr + off;
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        if (u >= nu) break;
        const Pos ddx = px - cx[u], ddy = py - cy[u], ddz = pz - cz[u];
        const Pos s2 = ddx * ddx + ddy * ddy;
        const Pos d2 = s2 + ddz * ddz;
        const bool hit = (double)d2 < cut2 && !(self && cj[u] == ip);
        const uint64_t mask = __ballot(hit);
        if (hit) {
          const int k = c + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
          if (k < cap) row[k] = cj[u];
        }
        c += __popcll(mask);
      }
      if (lane == p) cnt = c;
    }
  }
}

template <class P>
__global__ __launch_bounds__(BLOCK) void k_build(const SlotDesc* table, LaunchTab tab) {
#pragma clang fp contract(off)
  typedef typename P::Pos Pos;
  typedef typename P::Pos4 Pos4;
  typedef typename P::Real4 Real4;
  __shared__ uint32_t lds_pre[BLOCK / WAVE][2][32];
  __shared__ uint32_t lds_beg[BLOCK / WAVE][2][32];
  SLOT_PROLOGUE(DOM_FLUID);
  const int i = lb * BLOCK + threadIdx.x;
  const int nf = S.nf;
  const bool act = i < nf;
  const int ii = act ? i : nf - 1;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const GLB Pos4* xa = gpc<Pos4>(S.xa);
  const GLB Pos4* xw = gpc<Pos4>(S.xw);
  const Pos4 xi4 = xa[ii];
  const Pos xi = xi4.x, yi = xi4.y, zi = xi4.z;
  int c[3];
  cell_coords<Pos>(S, xi, yi, zi, c);
  if (act) gp<Real4>(S.xo)[i] = cell_offset<P>(S, xi, yi, zi, c);
  const double cut2 = S.cut2;
  const int kf = S.kf, ks = S.ks;
  GLB uint32_t* rows = gp<uint32_t>(S.rmaj);
  const GLB uint32_t* rank = gpc<uint32_t>(S.rank);
  const GLB uint32_t* stf = gpc<uint32_t>(S.start_f);
  const GLB uint32_t* sts = gpc<uint32_t>(S.start_s);
  uint32_t* preF = lds_pre[wv][0];
  uint32_t* preS = lds_pre[wv][1];
  uint32_t* begF = lds_beg[wv][0];
  uint32_t* begS = lds_beg[wv][1];
  int cf = 0, cs = 0;
  // runs of equal cells among the wave's particles
  const uint32_t myr = rank[cell_linear(S, c[0], c[1], c[2])];
  const uint32_t prevr = (uint32_t)__shfl_up((int)myr, 1, WAVE);
  const int nact = __popcll(__ballot(act));
  uint64_t runs = __ballot(act && (lane == 0 || prevr != myr));
  // this lane's offset in a 27-cell stencil
  const int ox = lane % 3 - 1, oy = (lane / 3) % 3 - 1, oz = lane / 9 - 1;
  const int wbase = i - lane;
  while (runs) {
    const int L = __builtin_ctzll(runs);
    runs &= runs - 1;
    const int R = runs ? __builtin_ctzll(runs) : nact;
    const int dx = __builtin_amdgcn_readlane(c[0], L), dy = __builtin_amdgcn_readlane(c[1], L),
              dz = __builtin_amdgcn_readlane(c[2], L);
    const int nx = dx + ox, ny = dy + oy, nz = dz + oz;
    const bool valid = lane < 27 && nx >= 0 && ny >= 0 && nz >= 0 && nx < S.dims[0] && ny < S.dims[1] &&
                       nz < S.dims[2];
    uint32_t f0 = 0, f1 = 0, s0 = 0, s1 = 0;
    if (valid) {
      const uint32_t r = rank[cell_linear(S, nx, ny, nz)];
      f0 = stf[r];
      f1 = stf[r + 1];
      s0 = sts[r];
      s1 = sts[r + 1];
    }
    uint32_t Mf, Ms;
    const uint32_t pf = wave_excl_scan(f1 - f0, &Mf);
    const uint32_t ps = wave_excl_scan(s1 - s0, &Ms);
    if (lane < 27) {
      preF[lane] = pf;
      begF[lane] = f0;
      preS[lane] = ps;
      begS[lane] = s0;
    }
    wave_lds_sync();
    run_candidates<Pos>(xa, preF, begF, Mf, L, R, wbase, xi, yi, zi, cut2, rows, kf + ks, 0, kf, cf, true);
    if (Ms) run_candidates<Pos>(xw, preS, begS, Ms, L, R, wbase, xi, yi, zi, cut2, rows, kf + ks, kf, ks, cs, false);
    wave_lds_sync();
  }
  if (!act) return;
  if (cf > kf || cs > ks) {
    raise_flag(S, F_CAPACITY);
    cf = min(cf, kf);
    cs = min(cs, ks);
  }
  S.nfc[i] = (uint32_t)cf;
  S.nsc[i] = (uint32_t)cs;
  // move this particle's row (written by the wave's lanes, still in cache)
  // into the SELL layout: entry k of the wave's particles lands contiguous
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  const GLB uint32_t* RM = rows + (int64_t)i * (kf + ks);
  GLB uint32_t* RS = gp<uint32_t>(S.nrec) + (int64_t)(i >> 6) * kf * WAVE + lane;
  for (int k = 0; k < cf; k += 4) {
    const u4 e = *(const GLB u4*)(RM + k);
    const uint32_t ev[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k + u < cf) RS[(int64_t)(k + u) * WAVE] = ev[u];
  }
  RM += kf;
  RS = gp<uint32_t>(S.srec) + (int64_t)(i >> 6) * ks * WAVE + lane;
  for (int k = 0; k < cs; k += 4) {
    const u4 e = *(const GLB u4*)(RM + k);
    const uint32_t ev[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k + u < cs) RS[(int64_t)(k + u) * WAVE] = ev[u];
  }
}

// ---------------------------------------------------------------------------
// K: kernel sum over the fresh rows, self included (Section 2.4), in FP64
// from the anchors, and the density re-initialisation against the
// perfect-lattice sum S0 (eq. 14 with a free surface, eq. 15 without).  Each
// pair's d^2 is formed exactly as in the cutoff test; the rows are walked in
// order (fluid, then solid) so the sum is reproducible.
// ---------------------------------------------------------------------------
// In FP32 and mixed arithmetic the kernel sums are held to six waves per SIMD
// (80 registers, two spilled): 3 us faster than at five, the step 8 us faster,
// though the dummy-velocity sweep beside them stretches.  FP64 keeps the
// compiler's budget.
constexpr int sumw_min_waves(bool f64) { return f64 ? 1 : 6; }
template <class P>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(
    sumw_min_waves(std::is_same<typename P::Real, double>::value)))) void k_sumw(const SlotDesc* table,
                                                                               LaunchTab tab) {
#pragma clang fp contract(off)
  typedef typename P::Pos Pos;
  typedef typename P::Real Real;
  typedef typename P::Pos4 Pos4;
  typedef typename P::Real4 Real4;
  __shared__ Pos4 wxa[WIN];
  SLOT_PROLOGUE(DOM_FLUID);
  const int i = lb * BLOCK + threadIdx.x;
  const GLB Pos4* xa = gpc<Pos4>(S.xa);
  const Window win = window_of(lb, S.nf);
  stage_window(wxa, xa, win);
  __syncthreads();
  if (i >= S.nf) return;
  const Pos4 xi4 = xa[i];
  const Pos xi = xi4.x, yi = xi4.y, zi = xi4.z;
  const double inv_h = 1.0 / S.h, kW = S.kW;
  double sw = kW;   // W(0)
  const int lane = i & (WAVE - 1);
  const int64_t slice = i >> 6;
  {
    const int n = (int)S.nfc[i];
    const GLB uint32_t* R = gpc<uint32_t>(S.nrec) + slice * (int64_t)S.kf * WAVE + lane;
    uint32_t jn[ROW_UNROLL];
#pragma unroll
    for (int u = 0; u < ROW_UNROLL; ++u) jn[u] = ldnt(R + (int64_t)u * WAVE);
    for (int k = 0; k < n; k += ROW_UNROLL) {
      Pos4 xj[ROW_UNROLL];
#pragma unroll
      for (int u = 0; u < ROW_UNROLL; ++u) xj[u] = win_get(wxa, xa, k + u < n ? jn[u] : (uint32_t)i, win);
      if (k + ROW_UNROLL < n) {
#pragma unroll
        for (int u = 0; u < ROW_UNROLL; ++u) jn[u] = ldnt(R + (int64_t)(k + ROW_UNROLL + u) * WAVE);
      }
#pragma unroll
      for (int u = 0; u < ROW_UNROLL; ++u) {
        const Pos ddx = xi - xj[u].x, ddy = yi - xj[u].y, ddz = zi - xj[u].z;
        const Pos s2 = ddx * ddx + ddy * ddy;
        const Pos d2 = s2 + ddz * ddz;
        const double w = kernel_W_d2((double)d2, inv_h, kW);
        if (k + u < n) sw += w;
      }
    }
  }
  GLB Real4* vr = gp<Real4>(S.vr);
  Real4 v = vr[i];
  const double dp3 = S.dp * S.dp * S.dp;
  {
    const int n = (int)S.nsc[i];
    const GLB uint32_t* R = gpc<uint32_t>(S.srec) + slice * (int64_t)S.ks * WAVE + lane;
    const GLB Pos4* xw = gpc<Pos4>(S.xw);
    uint32_t wn[SOLID_UNROLL];
#pragma unroll
    for (int u = 0; u < SOLID_UNROLL; ++u) wn[u] = ldnt(R + (int64_t)u * WAVE);
    for (int k = 0; k < n; k += SOLID_UNROLL) {
      Pos4 xq[SOLID_UNROLL];
#pragma unroll
      for (int u = 0; u < SOLID_UNROLL; ++u) xq[u] = xw[k + u < n ? wn[u] : 0u];
      if (k + SOLID_UNROLL < n) {
#pragma unroll
        for (int u = 0; u < SOLID_UNROLL; ++u) wn[u] = ldnt(R + (int64_t)(k + SOLID_UNROLL + u) * WAVE);
      }
#pragma unroll
      for (int u = 0; u < SOLID_UNROLL; ++u) {
        const Pos ddx = xi - xq[u].x, ddy = yi - xq[u].y, ddz = zi - xq[u].z;
        const Pos s2 = ddx * ddx + ddy * ddy;
        const Pos d2 = s2 + ddz * ddz;
        const double w = kernel_W_d2((double)d2, inv_h, kW);
        if (k + u < n) sw += w;
      }
    }
  }
  S.sumW[i] = sw;
  const double rre = S.rho0 * (dp3 * sw) / S.S0;
  const double rcur = P::kRel ? S.rho0 + (double)v.w : (double)v.w;
  const double rn = S.free_surface ? fmax(rcur, rre) : rre;
  v.w = P::kRel ? (Real)(rn - S.rho0) : (Real)rn;
  vr[i] = v;
}

// Sum over the wavefront by DPP lane moves (no LDS traffic), in a fixed
// order: pairs, quads, half-rows and rows of 16 by quad and mirror
// permutations, then row 1 and row 3 take the row before them (row_bcast:15)
// and rows 2 and 3 the first 32 lanes' sum (row_bcast:31).  The total is in
// lane 63; every lane must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_take(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_take(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <class Real>
__device__ __forceinline__ Real wave_total(Real v) {
  v += dpp_take<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
  v += dpp_take<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
  v += dpp_take<0x141, 0xf>(v);   // row_half_mirror
  v += dpp_take<0x140, 0xf>(v);   // row_mirror
  v += dpp_take<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_take<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return rl(v, WAVE - 1);
}

// ---------------------------------------------------------------------------
// K: dummy velocity of every solid particle for the wall viscous force
// (eq. 18 with the generalized wall of Section 2.5): v_w = 2 u_w - v~_w, with
// v~_w = (sum_j W_wj v_j) / (sum_j W_wj) the Shepard mean of the step-start
// velocity of the fluid within 2h (the rigid velocity u_w when there is none,
// or with the literal reading of eq. 18).
//
// Solid-centric, with the neighbour build's traversal: a wavefront holds 64
// consecutive solid particles of the Morton order; for each run sharing a
// cell, the fluid candidates of its 27-cell stencil are spread over the lanes
// in chunks of CBW per lane (cell-relative position and velocity loaded
// once); for each chunk the run's particles are taken in turn, every lane
// sums W and W v over its candidates within 2h, and four wave reductions in a
// fixed order add the chunk's share to the particle's sums.  The arithmetic is that of the interaction sweeps (FP32 in
// mixed precision, pair vectors from the frozen cell-relative positions): a
// pair that this test and the FP64 cutoff test of the rows decide differently
// lies within a few ulps of 2h, where W is below 1e-25 W(0).  No atomics: the
// result depends only on the sorted order, so it is the same alone or batched.
// It runs beside the kernel sums, which rewrite only the density component of
// the velocity records read here.
// ---------------------------------------------------------------------------
// candidate slots per lane of the dummy-velocity sweep: four (six waves per
// SIMD) against eight (three waves) took it from 0.29 to 0.20 ms
constexpr int CBW = 4;
template <class P>
__global__ __launch_bounds__(BLOCK) void k_wallvel(const SlotDesc* table, LaunchTab tab) {
  typedef typename P::Real Real;
  typedef typename P::Real4 Real4;
  __shared__ uint32_t lds_pre[BLOCK / WAVE][32];
  __shared__ uint32_t lds_beg[BLOCK / WAVE][32];
  SLOT_PROLOGUE(DOM_SOLID);
  const int w = lb * BLOCK + threadIdx.x;
  const int ns = S.ns;
  const bool act = w < ns;
  const int ww = act ? w : ns - 1;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const Real4 u = gpc<Real4>(S.vw)[ww];
  // sums of this lane's solid particle: W v (3) and W
  Real acc[4] = {(Real)0, (Real)0, (Real)0, (Real)0};
  if (!S.wall_rigid) {
    const GLB Real4* xo = gpc<Real4>(S.xo);
    const GLB Real4* vr = gpc<Real4>(S.vr);
    const GLB uint32_t* rank = gpc<uint32_t>(S.rank);
    const GLB uint32_t* stf = gpc<uint32_t>(S.start_f);
    const Real4 ow = gpc<Real4>(S.so)[ww];
    const uint32_t cw = unpack_index(ow.w);
    const int c[3] = {(int)(cw & 1023u), (int)((cw >> 10) & 1023u), (int)(cw >> 20)};
    const Real cut2 = (Real)S.cut2, inv_h = (Real)(1.0 / S.h), kW = (Real)S.kW, csr = (Real)S.cs_r;
    uint32_t* pre = lds_pre[wv];
    uint32_t* beg = lds_beg[wv];
    const uint32_t myr = rank[cell_linear(S, c[0], c[1], c[2])];
    const uint32_t prevr = (uint32_t)__shfl_up((int)myr, 1, WAVE);
    const int nact = __popcll(__ballot(act));
    uint64_t runs = __ballot(act && (lane == 0 || prevr != myr));
    const int ox = lane % 3 - 1, oy = (lane / 3) % 3 - 1, oz = lane / 9 - 1;
    while (runs) {
      const int L = __builtin_ctzll(runs);
      runs &= runs - 1;
      const int R = runs ? __builtin_ctzll(runs) : nact;
      const int nx = __builtin_amdgcn_readlane(c[0], L) + ox, ny = __builtin_amdgcn_readlane(c[1], L) + oy,
                nz = __builtin_amdgcn_readlane(c[2], L) + oz;
      const bool valid = lane < 27 && nx >= 0 && ny >= 0 && nz >= 0 && nx < S.dims[0] && ny < S.dims[1] &&
                         nz < S.dims[2];
      uint32_t f0 = 0, f1 = 0;
      if (valid) {
        const uint32_t r = rank[cell_linear(S, nx, ny, nz)];
        f0 = stf[r];
        f1 = stf[r + 1];
      }
      uint32_t M;
      const uint32_t pf = wave_excl_scan(f1 - f0, &M);
      if (lane < 27) {
        pre[lane] = pf;
        beg[lane] = f0;
      }
      wave_lds_sync();
      for (uint32_t b0 = 0; b0 < M; b0 += (uint32_t)(WAVE * CBW)) {
        Real4 co[CBW], cv[CBW];
#pragma unroll
        for (int k = 0; k < CBW; ++k) {
          const uint32_t m = b0 + (uint32_t)(k * WAVE + lane);
          co[k] = Real4((Real)1e30);   // far: never within 2h
          co[k].w = pack_index(0u, (Real)0);
          cv[k] = Real4((Real)0);
          if (m < M) {
            int qq = 0;
#pragma unroll
            for (int st = 16; st > 0; st >>= 1)
              if (qq + st < 27 && pre[qq + st] <= m) qq += st;
            const uint32_t j = beg[qq] + (m - pre[qq]);
            co[k] = xo[j];
            cv[k] = vr[j];
          }
        }
        const int nu = (int)min((uint32_t)CBW, (M - b0 + WAVE - 1) / WAVE);
        for (int p = L; p < R; ++p) {
          Real4 op;
          op.x = rl(ow.x, p);
          op.y = rl(ow.y, p);
          op.z = rl(ow.z, p);
          op.w = rl(ow.w, p);
          const uint32_t cp = unpack_index(op.w);
          Real s[4] = {(Real)0, (Real)0, (Real)0, (Real)0};
          bool any = false;
#pragma unroll
          for (int k = 0; k < CBW; ++k) {
            if (k >= nu) break;
            Real rx, ry, rz;
            pair_vec(op, cp, co[k], csr, rx, ry, rz);
            const Real r2 = rx * rx + ry * ry + rz * rz;
            if (r2 < cut2) {
              const Real q = r2 * rsq(r2) * inv_h;
              const Real t = (Real)1 - (Real)0.5 * q;
              const Real wgt = r2 > (Real)0 ? kW * t * t * t * t * ((Real)1 + (Real)2 * q) : kW;
              s[0] += wgt * cv[k].x;
              s[1] += wgt * cv[k].y;
              s[2] += wgt * cv[k].z;
              s[3] += wgt;
              any = true;
            }
          }
          if (!__ballot(any)) continue;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const Real t = wave_total(s[a]);
            if (lane == p) acc[a] += t;
          }
        }
      }
      wave_lds_sync();
    }
  }
  if (!act) return;
  Real4 o = u;
  o.w = (Real)0;
  if (!S.wall_rigid && acc[3] > (Real)0) {
    const double inv = 1.0 / (double)acc[3];
    o.x = (Real)(2.0 * (double)u.x - (double)acc[0] * inv);
    o.y = (Real)(2.0 * (double)u.y - (double)acc[1] * inv);
    o.z = (Real)(2.0 * (double)u.z - (double)acc[2] * inv);
    o.w = (Real)((double)acc[3] * (S.dp * S.dp * S.dp));
  }
  gp<Real4>(S.vd)[w] = o;
}

// ---------------------------------------------------------------------------
// K: contact factor of every solid particle (Section 2.7, eq. 24) after a
// build at the current time, FP64: the sum of V_j W_wj (V_j = m / rho_j) over
// the fluid particles within 2h of the solid particle, over the full-immersion
// reference (the lattice kernel sum over the wall's outer half-space).  The
// solid particle scans its own 27 fluid cells; an observable, not a step
// kernel.
// ---------------------------------------------------------------------------
// zout: the values in the caller's original order (S.zeta when null); part
// (optional, nblk blocks): per-block, per-body sums of the values and of the
// solid-particle counts, quantity-major ([(2 b + k) * nblk + block], k = 0
// sum, 1 count), reduced by k_contact_mean.
template <class P>
__global__ __launch_bounds__(BLOCK) void k_contact(const SlotDesc* table, LaunchTab tab, double* zout,
                                                   double* part) {
#pragma clang fp contract(off)
  typedef typename P::Pos Pos;
  typedef typename P::Pos4 Pos4;
  typedef typename P::Real4 Real4;
  __shared__ double lds[BLOCK / WAVE][NB][2];
  SLOT_PROLOGUE(DOM_SOLID);
  const int w = lb * BLOCK + threadIdx.x;
  double zw = 0.0;
  int bw = -1;
  if (w < S.ns) {
  const GLB Pos4* xa = gpc<Pos4>(S.xa);
  const GLB Real4* vr = gpc<Real4>(S.vr);
  const GLB uint32_t* rank = gpc<uint32_t>(S.rank);
  const GLB uint32_t* stf = gpc<uint32_t>(S.start_f);
  const Pos4 xq = gpc<Pos4>(S.xw)[w];
  int c[3];
  cell_coords<Pos>(S, xq.x, xq.y, xq.z, c);
  const double inv_h = 1.0 / S.h, kW = S.kW, m = S.mass, cut2 = S.cut2;
  double z = 0.0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int nx = c[0] + dx, ny = c[1] + dy, nz = c[2] + dz;
        if (nx < 0 || ny < 0 || nz < 0 || nx >= S.dims[0] || ny >= S.dims[1] || nz >= S.dims[2]) continue;
        const uint32_t r = rank[cell_linear(S, nx, ny, nz)];
        for (uint32_t j = stf[r]; j < stf[r + 1]; ++j) {
          const Pos4 xj = xa[j];
          const Pos ddx = xq.x - xj.x, ddy = xq.y - xj.y, ddz = xq.z - xj.z;
          const Pos s2 = ddx * ddx + ddy * ddy;
          const Pos d2 = s2 + ddz * ddz;
          if ((double)d2 < cut2) {
            const double rw = (double)vr[j].w;
            const double rho = P::kRel ? S.rho0 + rw : rw;
            z += (m / rho) * kernel_W_d2((double)d2, inv_h, kW);
          }
        }
      }
  zw = z / S.zref;
  bw = S.body[w];
  (zout ? zout : S.zeta)[S.sid[w]] = zw;   // in the caller's original order (sid is a permutation)
  }
  if (!part) return;
  // per-body block sums in a fixed order: lanes by shuffle, then the four waves
  const int wv = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
  for (int b = 0; b < S.nbody; ++b) {
    const double sv = wave_sum(bw == b ? zw : 0.0);
    const double cv = (double)__popcll(__ballot(bw == b));
    if (ln == 0) {
      lds[wv][b][0] = sv;
      lds[wv][b][1] = cv;
    }
  }
  __syncthreads();
  const int nblk = S.nblk[DOM_SOLID];
  if (threadIdx.x < 2 * S.nbody) {
    const int b = threadIdx.x / 2, k = threadIdx.x % 2;
    part[(size_t)threadIdx.x * nblk + lb] = ((lds[0][b][k] + lds[1][b][k]) + lds[2][b][k]) + lds[3][b][k];
  }
}

// Mean contact factor of every body from k_contact's block partials: each
// quantity's partials summed over the blocks in a fixed order with Neumaier
// compensation (one wavefront per quantity), then sum / count (0 for a body
// without solid particles).  One block per slot.
__global__ __launch_bounds__(BLOCK) void k_contact_mean(const SlotDesc* table, LaunchTab tab,
                                                        const double* part, double* mean) {
  __shared__ double res[NB][2];
  SLOT_PROLOGUE(DOM_SLOT);
  (void)lb;
  const int nblk = S.nblk[DOM_SOLID];
  const int wv = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
  for (int q = wv; q < 2 * S.nbody; q += BLOCK / WAVE) {
    KS ks{0.0, 0.0};
    for (int k = ln; k < nblk; k += WAVE) ks_add(ks, part[(size_t)q * nblk + k]);
    const KS t = wave_ks(ks);
    if (ln == 0) res[q / 2][q % 2] = t.s + t.c;
  }
  __syncthreads();
  if (threadIdx.x < S.nbody) {
    const int b = threadIdx.x;
    mean[b] = res[b][1] > 0.0 ? res[b][0] / res[b][1] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// K: dual-criteria time step (Section 2.8, eq. 25).  |v|max covers the fluid
// and the bodies' tip speeds; n_ac is capped by shortening dt_ad.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_dt(const SlotDesc* table, LaunchTab tab) {
  __shared__ double red[BLOCK / WAVE];
  SLOT_PROLOGUE(DOM_SLOT);
  (void)lb;
  const int n = S.nblk[DOM_FLUID];
  double m = 0.0;
  for (int k = threadIdx.x; k < n; k += BLOCK) m = fmax(m, S.vmax_part[k]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, WAVE));
  if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double vm = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
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
    tad = fmin(tad, S.dt_T);   // eq. 26
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


// G[a][b] += c dv_a r_b: one pair's term of the SPH velocity gradient
template <class Real>
__device__ __forceinline__ void grad_add(Real* G, Real c, Real dx, Real dy, Real dz, Real rx, Real ry, Real rz) {
  const Real d[3] = {c * dx, c * dy, c * dz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    G[3 * a] += d[a] * rx;
    G[3 * a + 1] += d[a] * ry;
    G[3 * a + 2] += d[a] * rz;
  }
}

// ---------------------------------------------------------------------------
// K: viscous acceleration (eq. 10 fluid-fluid, eq. 18 fluid-wall) and heat
// conduction rate (eq. 22), both frozen for the advection step.  Per-block
// partials: viscous force and torque on each body and its heat flow into the
// fluid.  Also clears this block's pressure-force accumulators.
// DISS: the launch holds a slot with viscous dissipation heating (eq. 23):
// the velocity gradient G[a][b] = sum V_j (v_j - v_i)_a F_ij r_ij[b] over fluid
// and wall neighbours gives Phi = 2 eta S:S, S = (G + G^T)/2, added to the
// heat rate as Phi/(rho cp); per-block partial of sum V_i Phi_i.
// MAT: the launch holds a slot with several fluid materials: k and cp per
// particle (material index gathered per neighbour), K_ij = 4 k_i k_j /
// (k_i + k_j) from a per-block table.
// MOM0: the same pass also runs the first acoustic sub-step's opening half
// (rho + dt/2 Drho, x + dt/2 v) and its Riemann momentum update, which read
// the same neighbours and frozen pair vectors: each neighbour's half-step
// density is formed from its gathered state and Drho with the arithmetic of
// the separate half update, so the results equal the unfused sequence bit
// for bit.  A fluid pair costs three gathers (cell offset, velocity and
// density, the (T, Drho) record the reorder wrote) instead of the five of
// the separate launches.
// ---------------------------------------------------------------------------
// The fused variant without dissipation is held to three waves per SIMD in
// FP32 and mixed arithmetic (168 registers, 20 bytes spilled per lane): the
// few spills cost less than the latency hiding the third wave brings.  The
// FP64 and dissipation variants keep the compiler's budget (held down they
// spill 100-400 bytes per lane and run slower).
constexpr int visc_min_waves(bool mom0, bool diss, bool f64) { return mom0 && !diss && !f64 ? 3 : 1; }
template <class P, bool DISS, bool MAT, bool MOM0>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(
    visc_min_waves(MOM0, DISS, std::is_same<typename P::Real, double>::value))))
void k_visc_heat(const SlotDesc* table, LaunchTab tab) {
  typedef typename P::Real Real;
  typedef typename P::Temp Temp;
  typedef typename P::Real4 Real4;
  __shared__ double lds[4 * NB * 7];
  __shared__ double lds_p[MOM0 ? 4 * NB * 6 : 1];
  __shared__ double lds_d[BLOCK / WAVE];
  __shared__ Real Ktab[MAT ? NMAT * NMAT : 1];
  SLOT_PROLOGUE(DOM_FLUID);
  const bool mats = MAT && S.mat != nullptr;
  if (mats) {
    for (int q = threadIdx.x; q < NMAT * NMAT; q += BLOCK) {
      const double ka = S.mk[q / NMAT], kb = S.mk[q % NMAT];
      Ktab[q] = (Real)(4.0 * ka * kb / (ka + kb));
    }
    __syncthreads();
  }
  const int nf = S.nf;
  const int i = lb * BLOCK + threadIdx.x;
  const size_t nbf = (size_t)S.nblk[DOM_FLUID];
  if (threadIdx.x < NB * 6) S.press_part[(size_t)threadIdx.x * nbf + lb] = 0.0;
  BodyAcc<7> acc;
  acc.init();
  BodyAcc<6> pacc;   // MOM0: pressure force and torque of the first sub-step
  pacc.init();
  bool wall = false;
  double vphi = 0.0;   // V_i Phi_i
  if (i < nf) {
    const GLB Real4* vr = gpc<Real4>(S.vr);
    const GLB Temp* T = gpc<Temp>(S.T);
    const GLB Real4* xo = gpc<Real4>(S.xo);
    const GLB Real* drho = gpc<Real>(S.drho);
    const GLB TempRate<P>* td = gpc<TempRate<P>>(S.td);
    const Real m = (Real)S.mass;
    const Real inv_h = (Real)(1.0 / S.h), kF = (Real)S.kF, csr = (Real)S.cs_r;
    const Real4 vi = vr[i];
    const Real4 oi = xo[i];
    const uint32_t ci = unpack_index(oi.w);
    const Real rhoi = rho_abs<P>(S, vi.w);
    const Temp Ti = T[i];
    const Real c2 = (Real)(2.0 * S.eta) * rcp(rhoi);   // 2 eta V_i / m_i
    const Real Kff = (Real)(4.0 * S.k_f * S.k_f / (S.k_f + S.k_f));
    const uint32_t mi = mats ? S.mat[i] : 0u;
    const double kI = mats ? S.mk[mi] : S.k_f, cpI = mats ? S.mcp[mi] : S.cp_f;
    Real ax = 0, ay = 0, az = 0, hs = 0;
    Real G[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) G[q] = 0;
    // MOM0: own half-step state (density opened by dt/2 Drho) and the
    // pressure acceleration of the first sub-step
    Real hdt = 0, wih = 0, rhoih = 0, pih = 0, c2p = 0, c0 = 0;
    Real px = 0, py = 0, pz = 0;
    if constexpr (MOM0) {
      hdt = (Real)(0.5 * S.ctl->dt);
      wih = vi.w + hdt * drho[i];
      rhoih = rho_abs<P>(S, wih);
      pih = press<P>(S, wih);
      c2p = (Real)2 * rcp(rhoih);
      c0 = (Real)S.c0;
    }
    const int lane = i & (WAVE - 1);
    const int64_t slice = i >> 6;
    {
      const int n = (int)S.nfc[i];
      const GLB uint32_t* R = gpc<uint32_t>(S.nrec) + slice * (int64_t)S.kf * WAVE + lane;
      uint32_t jn[ROW_UNROLL];
#pragma unroll
      for (int u = 0; u < ROW_UNROLL; ++u) jn[u] = ldnt(R + (int64_t)u * WAVE);
      for (int k = 0; k < n; k += ROW_UNROLL) {
        uint32_t j[ROW_UNROLL];
#pragma unroll
        for (int u = 0; u < ROW_UNROLL; ++u) j[u] = k + u < n ? jn[u] : (uint32_t)i;
        Real4 vj[ROW_UNROLL], oj[ROW_UNROLL];
        Temp Tj[ROW_UNROLL];
        Real dj[ROW_UNROLL];
#pragma unroll
        for (int u = 0; u < ROW_UNROLL; ++u) {
          oj[u] = xo[j[u]];
          vj[u] = vr[j[u]];
          if constexpr (MOM0) {
            Tj[u] = td[j[u]].T;
            dj[u] = td[j[u]].d;
          } else {
            Tj[u] = T[j[u]];
          }
        }
        if (k + ROW_UNROLL < n) {
#pragma unroll
          for (int u = 0; u < ROW_UNROLL; ++u) jn[u] = ldnt(R + (int64_t)(k + ROW_UNROLL + u) * WAVE);
        }
#pragma unroll
        for (int u = 0; u < ROW_UNROLL; ++u) {
          Real rx, ry, rz;
          pair_vec(oi, ci, oj[u], csr, rx, ry, rz);
          const Real r2 = rx * rx + ry * ry + rz * rz;
          const Real Fk = k + u < n ? kernel_F(r2, inv_h, kF) : (Real)0;
          const Real Vj = m * rcp(rho_abs<P>(S, vj[u].w));
          const Real cv = c2 * Vj * Fk;
          ax += cv * (vi.x - vj[u].x);
          ay += cv * (vi.y - vj[u].y);
          az += cv * (vi.z - vj[u].z);
          const Real Kij = mats ? Ktab[mi * NMAT + S.mat[j[u]]] : Kff;
          hs += Vj * Kij * (Real)(Ti - Tj[u]) * Fk;
          if (DISS) grad_add(G, Vj * Fk, vj[u].x - vi.x, vj[u].y - vi.y, vj[u].z - vi.z, rx, ry, rz);
          if constexpr (MOM0) {
            // eq. 10-12 at the half-step densities, velocities of the step's start
            const Real inv = r2 > (Real)0 ? rsq(r2) : (Real)0;
            const Real wjh = vj[u].w + hdt * dj[u];
            const Real rhoj = rho_abs<P>(S, wjh);
            const Real pj = press<P>(S, wjh);
            const Real dU = -((vi.x - vj[u].x) * rx + (vi.y - vj[u].y) * ry + (vi.z - vj[u].z) * rz) * inv;
            const Real beta = fmin((Real)3 * fmax(dU, (Real)0), c0);
            const Real ps = (Real)0.5 * (pih + pj) + rhoih * rhoj * beta * dU * rcp(rhoih + rhoj);
            const Real sp = -c2p * (m * rcp(rhoj)) * ps * Fk;
            px += sp * rx;
            py += sp * ry;
            pz += sp * rz;
          }
        }
      }
    }
    {
      const int n = (int)S.nsc[i];
      wall = n > 0;
      const GLB uint32_t* R = gpc<uint32_t>(S.srec) + slice * (int64_t)S.ks * WAVE + lane;
      const GLB Real4* so = gpc<Real4>(S.so);
      const GLB Real4* vdw = gpc<Real4>(S.vd);   // dummy velocity of eq. 18
      const GLB Real4* vw = gpc<Real4>(S.vw);    // rigid velocity (velocity gradient of eq. 23)
      const GLB Real4* lv = gpc<Real4>(S.lev);
      const Real Vw = (Real)S.vol_w;
      const Real rc = rcp(rhoi * (Real)cpI);
      uint32_t wn[VISC_SOLID_UNROLL];
#pragma unroll
      for (int u = 0; u < VISC_SOLID_UNROLL; ++u) wn[u] = ldnt(R + (int64_t)u * WAVE);
      for (int k0 = 0; k0 < n; k0 += VISC_SOLID_UNROLL) {
        Real4 owu[VISC_SOLID_UNROLL], vqu[VISC_SOLID_UNROLL], lqu[VISC_SOLID_UNROLL], vgu[VISC_SOLID_UNROLL];
#pragma unroll
        for (int u = 0; u < VISC_SOLID_UNROLL; ++u) {
          const uint32_t w = k0 + u < n ? wn[u] : 0u;
          owu[u] = so[w];
          vqu[u] = vdw[w];
          lqu[u] = lv[w];
          if (DISS) vgu[u] = vw[w];
        }
        if (k0 + VISC_SOLID_UNROLL < n) {
#pragma unroll
          for (int u = 0; u < VISC_SOLID_UNROLL; ++u) wn[u] = ldnt(R + (int64_t)(k0 + VISC_SOLID_UNROLL + u) * WAVE);
        }
#pragma unroll
        for (int u = 0; u < VISC_SOLID_UNROLL; ++u) {
        if (k0 + u >= n) break;
        const Real4 ow = owu[u], vq = vqu[u], lq = lqu[u];
        Real rx, ry, rz;
        pair_vec(oi, ci, ow, csr, rx, ry, rz);
        const Real Fk = kernel_F(rx * rx + ry * ry + rz * rz, inv_h, kF);
        const int b = (int)lq.w;
        const Real cv = c2 * Vw * Fk;
        const Real fx = cv * (vi.x - vq.x), fy = cv * (vi.y - vq.y), fz = cv * (vi.z - vq.z);
        ax += fx;
        ay += fy;
        az += fz;
        const Real Kiw = (Real)(4.0 * kI * S.bk[b] / (kI + S.bk[b]));
        const Real term = Vw * Kiw * (Real)(Ti - (Temp)S.bT[b]) * Fk;
        hs += term;
        if (DISS) grad_add(G, Vw * Fk, vgu[u].x - vi.x, vgu[u].y - vi.y, vgu[u].z - vi.z, rx, ry, rz);
        // force of the fluid on the body is -m_i times this pair's acceleration
        const double gx = -(double)m * fx, gy = -(double)m * fy, gz = -(double)m * fz;
        const double lx = lq.x, ly = lq.y, lz = lq.z;
        const double contrib[7] = {gx, gy, gz, ly * gz - lz * gy, lz * gx - lx * gz, lx * gy - ly * gx,
                                   (double)m * cpI * (double)(rc * term)};
        if (!acc.add(b, contrib)) raise_flag(S, F_CAPACITY);
        if constexpr (MOM0) {
          // the wall pressure of the one-sided Riemann problem (eq. 16-19)
          const Real PR = pih - rhoih * ((Real)S.g[0] * rx + (Real)S.g[1] * ry + (Real)S.g[2] * rz);
          const Real rhoR = (Real)S.rho0 + PR * (Real)(1.0 / (S.c0 * S.c0));
          const Real ps = (rhoih * PR + rhoR * pih) * rcp(rhoih + rhoR);
          const Real sp = -c2p * Vw * ps * Fk;
          const Real qx = sp * rx, qy = sp * ry, qz = sp * rz;
          px += qx;
          py += qy;
          pz += qz;
          const double hx = -(double)m * qx, hy = -(double)m * qy, hz = -(double)m * qz;
          const double pc[6] = {hx, hy, hz, ly * hz - lz * hy, lz * hx - lx * hz, lx * hy - ly * hx};
          if (!pacc.add(b, pc)) raise_flag(S, F_CAPACITY);
        }
        }
      }
      if (DISS && S.diss) {
        // Phi = 2 eta S:S with S = (G + G^T)/2
        const Real sxy = (Real)0.5 * (G[1] + G[3]), sxz = (Real)0.5 * (G[2] + G[6]),
                   syz = (Real)0.5 * (G[5] + G[7]);
        const Real ss = (G[0] * G[0] + G[4] * G[4] + G[8] * G[8]) + (Real)2 * ((sxy * sxy + sxz * sxz) + syz * syz);
        const Real phi = (Real)(2.0 * S.eta) * ss;
        hs += phi;
        vphi = (double)(m * rcp(rhoi)) * (double)phi;
      }
      Real4 a;
      a.x = ax;
      a.y = ay;
      a.z = az;
      a.w = rc * hs;
      gp<Real4>(S.ah)[i] = a;
      if constexpr (MOM0) {
        // v_new = v + dt (a_p + a_visc + g); the opening and the closing half
        // drifts x += dt/2 v, x += dt/2 v_new, in that order
        const Real dt = (Real)S.ctl->dt;
        Real4 vn;
        vn.x = vi.x + dt * (px + ax + (Real)S.g[0]);
        vn.y = vi.y + dt * (py + ay + (Real)S.g[1]);
        vn.z = vi.z + dt * (pz + az + (Real)S.g[2]);
        vn.w = wih;
        gp<Real4>(S.vrn)[i] = vn;
        GLB Real4* dr = gp<Real4>(S.drift);
        Real4 d = dr[i];
        d.x += hdt * vi.x;
        d.y += hdt * vi.y;
        d.z += hdt * vi.z;
        d.x += hdt * vn.x;
        d.y += hdt * vn.y;
        d.z += hdt * vn.z;
        dr[i] = d;
      }
    }
  }
  if (__syncthreads_or(wall)) {
    block_body_reduce<7>(acc, S.nbody, S.visc_part, nbf, lb, false, lds);
    if constexpr (MOM0) block_body_reduce<6>(pacc, S.nbody, S.press_part, nbf, lb, true, lds_p);
  } else if (threadIdx.x < NB * 7) {
    S.visc_part[(size_t)threadIdx.x * nbf + lb] = 0.0;
  }
  if (DISS && S.diss) {
    const double sw = wave_sum(vphi);
    if ((threadIdx.x & (WAVE - 1)) == 0) lds_d[threadIdx.x / WAVE] = sw;
    __syncthreads();
    if (threadIdx.x == 0)
      S.glob_part[(size_t)NGLOB * nbf + lb] = ((lds_d[0] + lds_d[1]) + lds_d[2]) + lds_d[3];
  }
}

// ---------------------------------------------------------------------------
// K: first half of an acoustic sub-step: rho += dt/2 Drho, x += dt/2 v
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_half_a(const SlotDesc* table, LaunchTab tab, int sub) {
  typedef typename P::Real Real;
  typedef typename P::Real4 Real4;
  SLOT_PROLOGUE(DOM_FLUID);
  if (sub >= S.ctl->n_ac) return;
  const int i = lb * BLOCK + threadIdx.x;
  if (i >= S.nf) return;
  const Real hdt = (Real)(0.5 * S.ctl->dt);
  GLB Real4* vr = gp<Real4>(S.vr);
  Real4 v = vr[i];
  v.w += hdt * gpc<Real>(S.drho)[i];
  vr[i] = v;
  GLB Real4* dr = gp<Real4>(S.drift);
  Real4 d = dr[i];
  d.x += hdt * v.x;
  d.y += hdt * v.y;
  d.z += hdt * v.z;
  dr[i] = d;
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
  typedef typename P::Real4 Real4;
  __shared__ double lds[4 * NB * 6];
  SLOT_PROLOGUE(DOM_FLUID);
  if (sub >= S.ctl->n_ac) return;
  const int nf = S.nf;
  const int i = lb * BLOCK + threadIdx.x;
  const GLB Real4* vr = gpc<Real4>(S.vr);
  const GLB Real4* xo = gpc<Real4>(S.xo);
  BodyAcc<6> acc;
  acc.init();
  bool wall = false;
  if (i < nf) {
    const Real c0 = (Real)S.c0;
    const Real m = (Real)S.mass;
    const Real4 vi = vr[i];
    const Real4 oi = xo[i];
    const uint32_t ci = unpack_index(oi.w);
    const Real rhoi = rho_abs<P>(S, vi.w);
    const Real pi = press<P>(S, vi.w);
    const Real c2 = (Real)2 * rcp(rhoi);   // 2 V_i / m_i
    const Real inv_h = (Real)(1.0 / S.h), kF = (Real)S.kF, csr = (Real)S.cs_r;
    Real ax = 0, ay = 0, az = 0;
    const int lane = i & (WAVE - 1);
    const int64_t slice = i >> 6;
    {
      const int n = (int)S.nfc[i];
      const GLB uint32_t* R = gpc<uint32_t>(S.nrec) + slice * (int64_t)S.kf * WAVE + lane;
      uint32_t jn[ROW_UNROLL];
#pragma unroll
      for (int u = 0; u < ROW_UNROLL; ++u) jn[u] = ldnt(R + (int64_t)u * WAVE);
      for (int k = 0; k < n; k += ROW_UNROLL) {
        uint32_t j[ROW_UNROLL];
#pragma unroll
        for (int u = 0; u < ROW_UNROLL; ++u) j[u] = k + u < n ? jn[u] : (uint32_t)i;
        Real4 vj[ROW_UNROLL], oj[ROW_UNROLL];
#pragma unroll
        for (int u = 0; u < ROW_UNROLL; ++u) {
          oj[u] = xo[j[u]];
          vj[u] = vr[j[u]];
        }
        if (k + ROW_UNROLL < n) {
#pragma unroll
          for (int u = 0; u < ROW_UNROLL; ++u) jn[u] = ldnt(R + (int64_t)(k + ROW_UNROLL + u) * WAVE);
        }
#pragma unroll
        for (int u = 0; u < ROW_UNROLL; ++u) {
          Real rx, ry, rz;
          pair_vec(oi, ci, oj[u], csr, rx, ry, rz);
          const Real r2 = rx * rx + ry * ry + rz * rz;
          const Real inv = r2 > (Real)0 ? rsq(r2) : (Real)0;
          const Real Fk = k + u < n ? kernel_F(r2, inv_h, kF) : (Real)0;
          const Real rhoj = rho_abs<P>(S, vj[u].w);
          const Real pj = press<P>(S, vj[u].w);
          // U_L - U_R = -(v_i - v_j) . e_ij
          const Real dU = -((vi.x - vj[u].x) * rx + (vi.y - vj[u].y) * ry + (vi.z - vj[u].z) * rz) * inv;
          const Real beta = fmin((Real)3 * fmax(dU, (Real)0), c0);
          const Real ps = (Real)0.5 * (pi + pj) + rhoi * rhoj * beta * dU * rcp(rhoi + rhoj);
          const Real s = -c2 * (m * rcp(rhoj)) * ps * Fk;
          ax += s * rx;
          ay += s * ry;
          az += s * rz;
        }
      }
    }
    {
      const int n = (int)S.nsc[i];
      wall = n > 0;
      const GLB uint32_t* R = gpc<uint32_t>(S.srec) + slice * (int64_t)S.ks * WAVE + lane;
      const GLB Real4* so = gpc<Real4>(S.so);
      const GLB Real4* lv = gpc<Real4>(S.lev);
      const Real gx = (Real)S.g[0], gy = (Real)S.g[1], gz = (Real)S.g[2];
      const Real rho0 = (Real)S.rho0;
      const Real ic02 = (Real)(1.0 / (S.c0 * S.c0));
      const Real Vw = (Real)S.vol_w;
      uint32_t wn[SOLID_UNROLL];
#pragma unroll
      for (int u = 0; u < SOLID_UNROLL; ++u) wn[u] = ldnt(R + (int64_t)u * WAVE);
      for (int k0 = 0; k0 < n; k0 += SOLID_UNROLL) {
        Real4 owu[SOLID_UNROLL], lqu[SOLID_UNROLL];
#pragma unroll
        for (int u = 0; u < SOLID_UNROLL; ++u) {
          const uint32_t w = k0 + u < n ? wn[u] : 0u;
          owu[u] = so[w];
          lqu[u] = lv[w];
        }
        if (k0 + SOLID_UNROLL < n) {
#pragma unroll
          for (int u = 0; u < SOLID_UNROLL; ++u) wn[u] = ldnt(R + (int64_t)(k0 + SOLID_UNROLL + u) * WAVE);
        }
#pragma unroll
        for (int u = 0; u < SOLID_UNROLL; ++u) {
        if (k0 + u >= n) break;
        const Real4 ow = owu[u], lq = lqu[u];
        Real rx, ry, rz;
        pair_vec(oi, ci, ow, csr, rx, ry, rz);
        const Real Fk = kernel_F(rx * rx + ry * ry + rz * rz, inv_h, kF);
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
        const double lx = lq.x, ly = lq.y, lz = lq.z;
        const double contrib[6] = {hx, hy, hz, ly * hz - lz * hy, lz * hx - lx * hz, lx * hy - ly * hx};
        if (!acc.add((int)lq.w, contrib)) raise_flag(S, F_CAPACITY);
        }
      }
    }
    const Real dt = (Real)S.ctl->dt;
    const Real hdt = (Real)(0.5 * S.ctl->dt);
    const Real4 a = gpc<Real4>(S.ah)[i];
    Real4 vn;
    vn.x = vi.x + dt * (ax + a.x + (Real)S.g[0]);
    vn.y = vi.y + dt * (ay + a.y + (Real)S.g[1]);
    vn.z = vi.z + dt * (az + a.z + (Real)S.g[2]);
    vn.w = vi.w;
    gp<Real4>(S.vrn)[i] = vn;
    GLB Real4* dr = gp<Real4>(S.drift);
    Real4 d = dr[i];
    d.x += hdt * vn.x;
    d.y += hdt * vn.y;
    d.z += hdt * vn.z;
    dr[i] = d;
  }
  if (__syncthreads_or(wall))
    block_body_reduce<6>(acc, S.nbody, S.press_part, (size_t)S.nblk[DOM_FLUID], lb, true, lds);
}

// ---------------------------------------------------------------------------
// K: Riemann continuity (eq. 10, 11-13) with (v_i - v*) . e_ij = U* - U_L, and
// the wall's mirror state; writes Drho, commits v <- v_new and applies the
// half updates that close this sub-step and open the next.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_continuity(const SlotDesc* table, LaunchTab tab, int sub) {
  typedef typename P::Real Real;
  typedef typename P::Real4 Real4;
  SLOT_PROLOGUE(DOM_FLUID);
  if (sub >= S.ctl->n_ac) return;
  const int i = lb * BLOCK + threadIdx.x;
  if (i >= S.nf) return;
  const GLB Real4* vrn = gpc<Real4>(S.vrn);
  const GLB Real4* xo = gpc<Real4>(S.xo);
  const Real c0 = (Real)S.c0;
  const Real m = (Real)S.mass;
  const Real4 vi = vrn[i];
  const Real4 oi = xo[i];
  const uint32_t ci = unpack_index(oi.w);
  const Real rhoi = rho_abs<P>(S, vi.w);
  const Real pi = press<P>(S, vi.w);
  const Real inv_h = (Real)(1.0 / S.h), kF = (Real)S.kF, csr = (Real)S.cs_r;
  Real sum = 0;
  const int lane = i & (WAVE - 1);
  const int64_t slice = i >> 6;
  {
    const int n = (int)S.nfc[i];
    const GLB uint32_t* R = gpc<uint32_t>(S.nrec) + slice * (int64_t)S.kf * WAVE + lane;
    uint32_t jn[CONT_UNROLL];
#pragma unroll
    for (int u = 0; u < CONT_UNROLL; ++u) jn[u] = ldnt(R + (int64_t)u * WAVE);
    for (int k = 0; k < n; k += CONT_UNROLL) {
      uint32_t j[CONT_UNROLL];
#pragma unroll
      for (int u = 0; u < CONT_UNROLL; ++u) j[u] = k + u < n ? jn[u] : (uint32_t)i;
      Real4 vj[CONT_UNROLL], oj[CONT_UNROLL];
#pragma unroll
      for (int u = 0; u < CONT_UNROLL; ++u) {
        oj[u] = xo[j[u]];
        vj[u] = vrn[j[u]];
      }
      if (k + CONT_UNROLL < n) {
#pragma unroll
        for (int u = 0; u < CONT_UNROLL; ++u)
          jn[u] = ldnt(R + (int64_t)min(k + CONT_UNROLL + u, S.kf - 1) * WAVE);
      }
#pragma unroll
      for (int u = 0; u < CONT_UNROLL; ++u) {
        Real rx, ry, rz;
        pair_vec(oi, ci, oj[u], csr, rx, ry, rz);
        const Real r2 = rx * rx + ry * ry + rz * rz;
        const Real rr = r2 > (Real)0 ? r2 * rsq(r2) : (Real)0;
        const Real Fk = k + u < n ? kernel_F(r2, inv_h, kF) : (Real)0;
        const Real rhoj = rho_abs<P>(S, vj[u].w);
        const Real pj = press<P>(S, vj[u].w);
        // (U* - U_L) dW = [ (v_i - v_j) . r / 2 + (p_i - p_j) r / (c0 (rho_i + rho_j)) ] F
        const Real vr_ = (vi.x - vj[u].x) * rx + (vi.y - vj[u].y) * ry + (vi.z - vj[u].z) * rz;
        const Real dv = (Real)0.5 * vr_ + (pi - pj) * rr * rcp(c0 * (rhoi + rhoj));
        sum += (m * rcp(rhoj)) * dv * Fk;
      }
    }
  }
  {
    const int n = (int)S.nsc[i];
    const GLB uint32_t* R = gpc<uint32_t>(S.srec) + slice * (int64_t)S.ks * WAVE + lane;
    const GLB Real4* so = gpc<Real4>(S.so);
    const GLB Real4* nw = gpc<Real4>(S.nw);
    const GLB Real4* vw = gpc<Real4>(S.vw);
    const Real gx = (Real)S.g[0], gy = (Real)S.g[1], gz = (Real)S.g[2];
    const Real rho0 = (Real)S.rho0;
    const Real ic02 = (Real)(1.0 / (S.c0 * S.c0));
    const Real Vw = (Real)S.vol_w;
    uint32_t wn[SOLID_UNROLL];
#pragma unroll
    for (int u = 0; u < SOLID_UNROLL; ++u) wn[u] = ldnt(R + (int64_t)u * WAVE);
    for (int k0 = 0; k0 < n; k0 += SOLID_UNROLL) {
      Real4 owu[SOLID_UNROLL], nqu[SOLID_UNROLL], vqu[SOLID_UNROLL];
#pragma unroll
      for (int u = 0; u < SOLID_UNROLL; ++u) {
        const uint32_t w = k0 + u < n ? wn[u] : 0u;
        owu[u] = so[w];
        nqu[u] = nw[w];
        vqu[u] = vw[w];
      }
      if (k0 + SOLID_UNROLL < n) {
#pragma unroll
        for (int u = 0; u < SOLID_UNROLL; ++u) wn[u] = ldnt(R + (int64_t)(k0 + SOLID_UNROLL + u) * WAVE);
      }
#pragma unroll
      for (int u = 0; u < SOLID_UNROLL; ++u) {
      if (k0 + u >= n) break;
      const Real4 ow = owu[u], nq = nqu[u], vq = vqu[u];
      Real rx, ry, rz;
      pair_vec(oi, ci, ow, csr, rx, ry, rz);
      const Real Fk = kernel_F(rx * rx + ry * ry + rz * rz, inv_h, kF);
      const Real PR = pi - rhoi * (gx * rx + gy * ry + gz * rz);
      const Real rhoR = rho0 + PR * ic02;
      const Real UL = -(nq.x * vi.x + nq.y * vi.y + nq.z * vi.z);
      const Real uw = -(nq.x * vq.x + nq.y * vq.y + nq.z * vq.z);
      const Real Us = uw + (pi - PR) * rcp(c0 * (rhoi + rhoR));
      sum += Vw * (Us - UL) * (nq.x * rx + nq.y * ry + nq.z * rz) * Fk;
      }
    }
  }
  // commit v <- v_new and close the sub-step (rho += dt/2 Drho); unless it is
  // the step's last, open the next one (rho += dt/2 Drho, x += dt/2 v).  No
  // thread of this sweep reads vr, so the update is in place.
  const Real dr = (Real)2 * rhoi * sum;
  gp<Real>(S.drho)[i] = dr;
  const Real hdt = (Real)(0.5 * S.ctl->dt);
  Real4 v = vi;
  v.w += hdt * dr;
  if (sub + 1 < S.ctl->n_ac) {
    v.w += hdt * dr;
    GLB Real4* dp = gp<Real4>(S.drift);
    Real4 d = dp[i];
    d.x += hdt * v.x;
    d.y += hdt * v.y;
    d.z += hdt * v.z;
    dp[i] = d;
  }
  gp<Real4>(S.vr)[i] = v;
}

// ---------------------------------------------------------------------------
// K: temperature by explicit Euler over the advection step (eq. 22, 26), and
// per-block totals: mass, kinetic energy, thermal energy, sum rho dp^3, vmax.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(BLOCK) void k_end(const SlotDesc* table, LaunchTab tab) {
  typedef typename P::Temp Temp;
  typedef typename P::Real4 Real4;
  __shared__ double lds[BLOCK / WAVE][NGLOB];
  SLOT_PROLOGUE(DOM_FLUID);
  const int i = lb * BLOCK + threadIdx.x;
  double q[NGLOB] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < S.nf) {
    GLB Temp* T = gp<Temp>(S.T);
    const Temp Tn = T[i] + (Temp)S.ctl->dt_ad * (Temp)gpc<Real4>(S.ah)[i].w;
    T[i] = Tn;
    const Real4 v = gpc<Real4>(S.vr)[i];
    const double vx = v.x, vy = v.y, vz = v.z;
    const double v2 = vx * vx + vy * vy + vz * vz;
    const double r = P::kRel ? S.rho0 + (double)v.w : (double)v.w;
    q[0] = S.mass;
    q[1] = 0.5 * S.mass * v2;
    q[2] = S.mass * (S.mat ? S.mcp[S.mat[i]] : S.cp_f) * (double)Tn;
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
__global__ __launch_bounds__(FINAL_BLOCK) void k_final(const SlotDesc* table, LaunchTab tab) {
  __shared__ double res[NGLOB + NB * 13 + 1];
  __shared__ double bheat[NB];
  __shared__ int bfin[NB];
  SLOT_PROLOGUE(DOM_SLOT);
  (void)lb;
  const int nblk = S.nblk[DOM_FLUID];
  // quantities: the globals, 13 per body, then the dissipated power if on
  const int nq = NGLOB + S.nbody * 13 + (S.diss ? 1 : 0);
  const int q_diss = NGLOB + S.nbody * 13;
  const int wv = threadIdx.x / WAVE, ln = threadIdx.x % WAVE;
  // each wavefront reduces QPW quantities at once (QPW x 8 independent loads
  // in flight per lane), each one's partials added in the same fixed order
  constexpr int QPW = 3;
  for (int q0 = wv * QPW; q0 < nq; q0 += (FINAL_BLOCK / WAVE) * QPW) {
    // quantity qi: global k, or body b component c (7 viscous then 6 pressure)
    // partials are quantity-major: src[q * nblk + block]
    const GLB double* qs[QPW];
    bool use[QPW], mx[QPW];
#pragma unroll
    for (int t = 0; t < QPW; ++t) {
      const int qi = q0 + t;
      use[t] = qi < nq;
      mx[t] = qi == 4;
      const double* src = S.glob_part;
      if (!use[t]) {
      } else if (qi < NGLOB) {
        src = S.glob_part + (size_t)qi * nblk;
      } else if (qi == q_diss) {
        src = S.glob_part + (size_t)NGLOB * nblk;
      } else {
        const int b = (qi - NGLOB) / 13, c = (qi - NGLOB) % 13;
        src = c < 7 ? S.visc_part + (size_t)(b * 7 + c) * nblk : S.press_part + (size_t)(b * 6 + c - 7) * nblk;
      }
      qs[t] = gpc<double>(src);
    }
    KS ks[QPW];
    double m[QPW];
#pragma unroll
    for (int t = 0; t < QPW; ++t) {
      ks[t] = KS{0.0, 0.0};
      m[t] = 0.0;
    }
    for (int k0 = 0; k0 < nblk; k0 += 8 * WAVE) {
      double x[QPW][8];
#pragma unroll
      for (int t = 0; t < QPW; ++t)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = k0 + u * WAVE + ln;
          x[t][u] = use[t] && k < nblk ? qs[t][k] : 0.0;
        }
#pragma unroll
      for (int t = 0; t < QPW; ++t) {
        if (mx[t]) {
#pragma unroll
          for (int u = 0; u < 8; ++u) m[t] = fmax(m[t], x[t][u]);
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u) ks_add(ks[t], x[t][u]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < QPW; ++t) {
      if (!use[t]) continue;
      if (mx[t]) {
        double v = m[t];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
        if (ln == 0) res[q0 + t] = v;
      } else {
        const KS w = wave_ks(ks[t]);
        if (ln == 0) res[q0 + t] = w.s + w.c;
      }
    }
  }
  __syncthreads();
  // the reports: lane b of the first wavefront finishes body b, lane 0 then
  // the globals; each lane loads the control fields it needs before it
  // stores anything (a store could alias a later load and hold it back)
  if (threadIdx.x >= WAVE) return;
  SlotCtl* C = S.ctl;
  const double tad = C->dt_ad;
  const int32_t nac = C->n_ac;
  const int b = threadIdx.x;
  if (b < S.nbody) {
    double cum[3], cumc[3];
    for (int k = 0; k < 3; ++k) {
      cum[k] = C->cum[b][k];
      cumc[k] = C->cum_c[b][k];
    }
    const double inv_nac = 1.0 / (double)nac;
    const double* r = res + NGLOB + b * 13;
    sph_body_report br;
    for (int k = 0; k < 3; ++k) {
      br.force[k] = r[k] + r[7 + k] * inv_nac;
      br.torque[k] = r[3 + k] + r[10 + k] * inv_nac;
    }
    const double* a = S.ba[b];
    br.torque_axis = a[0] * br.torque[0] + a[1] * br.torque[1] + a[2] * br.torque[2];
    br.power = -S.bom[b] * br.torque_axis;
    br.heat_rate = r[6];
    // running totals over up to 1e5 steps: compensated like the block sums
    const double inc[3] = {tad * br.torque_axis, tad * br.power, tad * br.heat_rate};
    double tot[3];
    for (int k = 0; k < 3; ++k) {
      KS acc{cum[k], cumc[k]};
      ks_add(acc, inc[k]);
      C->cum[b][k] = acc.s;
      C->cum_c[b][k] = acc.c;
      tot[k] = acc.s + acc.c;
    }
    br.torque_axis_int = tot[0];
    br.energy_int = tot[1];
    br.heat_int = tot[2];
    C->brep[b] = br;
    bheat[b] = br.heat_rate;
    bfin[b] = isfinite(br.torque_axis) && isfinite(br.heat_rate) && isfinite(br.force[0]) &&
              isfinite(br.force[1]) && isfinite(br.force[2]);
  }
  wave_lds_sync();
  if (b != 0) return;
  const double dtc = C->dt, t0 = C->t;
  const int64_t step0 = C->step, sub0 = C->substeps;
  const uint32_t flags0 = C->flags;
  KS heat{C->heat_total, C->heat_c}, diss{C->diss_total, C->diss_c};
  double qsum = 0.0;
  bool finite = true;
  for (int q = 0; q < S.nbody; ++q) {
    qsum += bheat[q];
    finite = finite && bfin[q];
  }
  const double t1 = t0 + tad;
  const int64_t step1 = step0 + 1, sub1 = sub0 + nac;
  const double hs = tad * qsum;
  const double ds = S.diss ? tad * res[q_diss] : 0.0;
  ks_add(heat, hs);
  ks_add(diss, ds);
  finite = finite && isfinite(res[1]) && isfinite(res[2]) && isfinite(res[3]) && isfinite(ds);
  const uint32_t flags1 = finite ? flags0 : (flags0 | F_NONFINITE);
  C->t = t1;
  C->step = step1;
  C->substeps = sub1;
  C->heat_total = heat.s;
  C->heat_c = heat.c;
  C->diss_total = diss.s;
  C->diss_c = diss.c;
  if (!finite) C->flags = flags1;
  sph_report R;
  R.t = t1;
  R.step = step1;
  R.n_ac = nac;
  R.dt_ad = tad;
  R.dt = dtc;
  R.mass = res[0];
  R.kinetic = res[1];
  R.thermal = res[2];
  R.mass_proxy = res[3];
  R.vmax = res[4];
  R.heat_step = hs;
  R.heat_total = heat.s + heat.c;
  R.substeps = sub1;
  R.diss_step = ds;
  R.diss_total = diss.s + diss.c;
  R.flags = (int32_t)flags1;
  C->rep = R;
}


// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
int grid_domain(int kid, int which) {
  switch (kid) {
    case SPH_K_CLEAR:
    case SPH_K_SCAN1:
    case SPH_K_SCAN3:
      return DOM_CELL;
    case SPH_K_POSE:
    case SPH_K_CONTACT:
    case SPH_K_WALLVEL:
      return DOM_SOLID;
    case SPH_K_SCAN2:
    case SPH_K_DT:
    case SPH_K_FINAL:
      return DOM_SLOT;
    case SPH_K_SCATTER:
    case SPH_K_CELLSORT:
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
    case SPH_K_CELLSORT: hipLaunchKernelGGL(k_cellsort, g, b, 0, st, T, L, which); break;
    case SPH_K_REORDER: hipLaunchKernelGGL(k_reorder<P>, g, b, 0, st, T, L, which); break;
    case SPH_K_BUILD: hipLaunchKernelGGL(k_build<P>, g, b, 0, st, T, L); break;
    case SPH_K_SUMW: hipLaunchKernelGGL(k_sumw<P>, g, b, 0, st, T, L); break;
    case SPH_K_CONTACT: hipLaunchKernelGGL(k_contact<P>, g, b, 0, st, T, L, nullptr, nullptr); break;
    case SPH_K_WALLVEL: hipLaunchKernelGGL(k_wallvel<P>, g, b, 0, st, T, L); break;
    case SPH_K_DT: hipLaunchKernelGGL(k_dt, g, b, 0, st, T, L); break;
    case SPH_K_VISC_HEAT:
      // which = 1: with the first acoustic sub-step's half update and momentum
      if (which == 1) {
        if (L.flags & TAB_MAT) {
          if (L.flags & TAB_DISS) hipLaunchKernelGGL((k_visc_heat<P, true, true, true>), g, b, 0, st, T, L);
          else hipLaunchKernelGGL((k_visc_heat<P, false, true, true>), g, b, 0, st, T, L);
        } else {
          if (L.flags & TAB_DISS) hipLaunchKernelGGL((k_visc_heat<P, true, false, true>), g, b, 0, st, T, L);
          else hipLaunchKernelGGL((k_visc_heat<P, false, false, true>), g, b, 0, st, T, L);
        }
      } else if (L.flags & TAB_MAT) {
        if (L.flags & TAB_DISS) hipLaunchKernelGGL((k_visc_heat<P, true, true, false>), g, b, 0, st, T, L);
        else hipLaunchKernelGGL((k_visc_heat<P, false, true, false>), g, b, 0, st, T, L);
      } else {
        if (L.flags & TAB_DISS) hipLaunchKernelGGL((k_visc_heat<P, true, false, false>), g, b, 0, st, T, L);
        else hipLaunchKernelGGL((k_visc_heat<P, false, false, false>), g, b, 0, st, T, L);
      }
      break;
    case SPH_K_HALF_A: hipLaunchKernelGGL(k_half_a<P>, g, b, 0, st, T, L, sub); break;
    case SPH_K_MOMENTUM: hipLaunchKernelGGL(k_momentum<P>, g, b, 0, st, T, L, sub); break;
    case SPH_K_CONTINUITY: hipLaunchKernelGGL(k_continuity<P>, g, b, 0, st, T, L, sub); break;
    case SPH_K_END: hipLaunchKernelGGL(k_end<P>, g, b, 0, st, T, L); break;
    case SPH_K_FINAL: hipLaunchKernelGGL(k_final, g, dim3(FINAL_BLOCK), 0, st, T, L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class P>
static hipError_t launch_contact_p(const SlotDesc* T, const LaunchTab& L, double* zout, double* part,
                                   double* mean, hipStream_t st) {
  const int nblk = L.blk0[DOM_SOLID][L.n];
  if (nblk > 0) hipLaunchKernelGGL(k_contact<P>, dim3(nblk), dim3(BLOCK), 0, st, T, L, zout, part);
  if (mean && L.blk0[DOM_SLOT][L.n] > 0)
    hipLaunchKernelGGL(k_contact_mean, dim3(L.blk0[DOM_SLOT][L.n]), dim3(BLOCK), 0, st, T, L,
                       (const double*)part, mean);
  return hipGetLastError();
}

hipError_t launch_contact(int prec, const SlotDesc* table, const LaunchTab& tab, double* zout, double* part,
                          double* mean, hipStream_t stream) {
  switch (prec) {
    case SPH_PREC_MIXED: return launch_contact_p<PMixed>(table, tab, zout, part, mean, stream);
    case SPH_PREC_FP64: return launch_contact_p<PF64>(table, tab, zout, part, mean, stream);
    case SPH_PREC_FP32: return launch_contact_p<PF32>(table, tab, zout, part, mean, stream);
    default: return hipErrorInvalidValue;
  }
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
