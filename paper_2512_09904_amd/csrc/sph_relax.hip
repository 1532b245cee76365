// sph_relax.hip -- physics-driven particle relaxation (arXiv 2512.09904,
// Section 2.2, eq. 5-9) on gfx950: FP64 level sets of analytic shapes, the
// relaxation force over the neighbour rows of the solver's own cell sort and
// build, and the move with level-set confinement.  Launched by sph_relax; one
// iteration is sort/build -> relax_force -> relax_max -> relax_move.
#include <algorithm>
#include <mutex>
#include <vector>

#include "sph_device.h"

namespace sphk {

// Cells of the exterior-integral quadrature: the cube [-2h, 2h]^3 cut into
// 16^3 cells of edge h/4, cell (a, b, c) centred at (a + 1/2, b + 1/2, c + 1/2)
// h/4 from the particle, a, b, c in [-8, 8).  They are visited by blocks of
// 2 x 2 x 2 cells: block (A, B, C), A, B, C in [-4, 4), holds the cells
// a in {2A, 2A + 1} (and likewise b, c), its centre at (2A + 1, 2B + 1, 2C + 1)
// h/4, every cell centre within sqrt(3)/2 h/4 of it.  Only blocks with key
// (2A+1)^2 + (2B+1)^2 + (2C+1)^2 = (distance / (h/4))^2 below 81 can hold a
// cell within 2h (8 h/4) of the particle; they are listed by ascending key
// (ties by linear index), so the blocks nearer than a distance form a prefix.
// Entry: key << 12 | (A+4) << 8 | (B+4) << 4 | (C+4).
constexpr int QK = 8, QKEY_MAX = 81, QMAX = 512;
// workgroups per block of particles in the force kernel, and the first row
// of the per-block partials that holds their maxima (rows RELAX_ROW to
// RELAX_ROW + RQ - 1, free between advection steps)
constexpr int RQ = 4, RELAX_ROW = NGLOB + 1 - RQ;
static_assert(RQ == BLOCK / WAVE && RELAX_ROW >= 0, "one integrating wavefront per residue of the lane");
constexpr double QHALFDIAG = 0.87;   // >= sqrt(3)/2: cell centre to block centre, in units of h/4
__constant__ uint32_t qcells[QMAX];

static int qcells_count = 0;
static bool qcells_loaded[64] = {};

// the table, built on the host and copied to the current device once (under
// a lock: solvers on different host threads may start a relaxation together)
static std::mutex qcells_mutex;
static hipError_t qcells_init(int* count) {
  std::lock_guard<std::mutex> lock(qcells_mutex);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (!qcells_loaded[dev]) {
    std::vector<uint64_t> v;
    const int BK = QK / 2;
    for (int a = -BK; a < BK; ++a)
      for (int b = -BK; b < BK; ++b)
        for (int c = -BK; c < BK; ++c) {
          const uint32_t key = (uint32_t)((2 * a + 1) * (2 * a + 1) + (2 * b + 1) * (2 * b + 1) + (2 * c + 1) * (2 * c + 1));
          if (key >= (uint32_t)QKEY_MAX) continue;
          const uint32_t lin = (uint32_t)(((a + BK) * QK + (b + BK)) * QK + (c + BK));
          const uint32_t ent = key << 12 | (uint32_t)(a + BK) << 8 | (uint32_t)(b + BK) << 4 | (uint32_t)(c + BK);
          v.push_back((uint64_t)key << 44 | (uint64_t)lin << 32 | ent);
        }
    std::sort(v.begin(), v.end());
    if ((int)v.size() > QMAX) return hipErrorInvalidValue;
    std::vector<uint32_t> t(v.size());
    for (size_t k = 0; k < v.size(); ++k) t[k] = (uint32_t)v[k];
    e = hipMemcpyToSymbol(HIP_SYMBOL(qcells), t.data(), t.size() * sizeof(uint32_t));
    if (e != hipSuccess) return e;
    qcells_count = (int)t.size();
    qcells_loaded[dev] = true;
  }
  *count = qcells_count;
  return hipSuccess;
}

// Every level-set evaluation is FP64.

// LDS written by some lanes of a wavefront, then read by others
__device__ __forceinline__ void relax_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// signed distance of the extrusion along y (|y| <= half) of a cross-section
// with signed distance d2
__device__ double ls_extrude(double d2, double y, double half) {
  const double dy = fabs(y) - half;
  const double ox = fmax(d2, 0.0), oy = fmax(dy, 0.0);
  return sqrt(ox * ox + oy * oy) + fmin(fmax(d2, dy), 0.0);
}

// Directions of the gear's flanks: entry j (0 <= j < 2 teeth) is the unit
// vector at the angle of tooth coordinate j/2, theta_j = 2 pi (j/2 - 1/4 -
// phase) / teeth.  Every block computes the table into LDS once.
constexpr int MAX_TEETH = 512;
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ void ls_flank_table(const RelaxShape& g, d2v* E) {
  if (g.kind != SPH_SHAPE_GEAR) return;
  for (int j = threadIdx.x; j < 2 * g.teeth; j += blockDim.x) {
    double sn, cs;
    sincos(2.0 * M_PI * (0.5 * (double)j - 0.25 - g.phase) / (double)g.teeth, &sn, &cs);
    E[j] = d2v{cs, sn};
  }
}

// squared distance from (px, pz) to the radial segment along e from r_root
// to r_tip
__device__ __forceinline__ double ls_flank2(const RelaxShape& g, double px, double pz, d2v e) {
  const double t = fmin(fmax(px * e.x + pz * e.y, g.size[1]), g.size[0]);
  const double ex = px - t * e.x, ez = pz - t * e.y;
  return ex * ex + ez * ez;
}

// Gear cross-section: root disk plus teeth where frac(u) < 1/2, u = z theta /
// 2 pi + 1/4 + phase.  Boundary: tip arcs over teeth, root arcs over gaps and
// radial flanks at half-integer u; the nearest piece belongs to the point's
// half-pitch k = floor(2u) or one of its two neighbours: flanks k-1 .. k+2,
// the own arc (radial distance) and the neighbours' arcs (their end points).
// The point distances are compared squared and rooted once: sqrt is
// correctly rounded and monotonic, so this is the minimum of their roots.
__device__ __forceinline__ void ls_sector(const d2v* E, int n2, int k, d2v e[4]) {
  // phase in [0, 1) keeps k in [-teeth - 1, teeth + 3]: one wrap each way
  int j0 = k - 1;
  j0 += j0 < 0 ? n2 : 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int j = j0 + m;
    e[m] = E[min(max(j >= n2 ? j - n2 : j, 0), n2 - 1)];   // the clamp only guards a non-finite point
  }
}

__device__ double ls_gear2d(const RelaxShape& g, const d2v* E, double px, double pz) {
  const double r = sqrt(px * px + pz * pz);
  const int n2 = 2 * g.teeth;
  // half-pitch k = floor(2u), u = zu theta + 1/4 + phase (zu = teeth / 2 pi):
  // estimated from an FP32 angle, then settled by the sides of its flanks
  // (the point lies in half-pitch k when it is on or left of flank k and
  // right of flank k + 1)
  const double ue = g.zu * (double)atan2f((float)pz, (float)px) + 0.25 + g.phase;
  int k = (int)floor(2.0 * ue);
  d2v e[4];
  ls_sector(E, n2, k, e);
  if (e[1].x * pz - e[1].y * px < 0.0) {
    k -= 1;
    ls_sector(E, n2, k, e);
  } else if (e[2].x * pz - e[2].y * px >= 0.0) {
    k += 1;
    ls_sector(E, n2, k, e);
  }
  double b2 = INFINITY;
#pragma unroll
  for (int m = 0; m < 4; ++m) b2 = fmin(b2, ls_flank2(g, px, pz, e[m]));
  // tip arc over a tooth (even half-pitch), root arc over a gap
  const bool even = (k & 1) == 0;
  const double Rn = even ? g.size[1] : g.size[0];   // the neighbours' arcs
#pragma unroll
  for (int m = 0; m < 4; ++m) {                     // their end points: flanks k-1 .. k+2
    const double ax = px - Rn * e[m].x, az = pz - Rn * e[m].y;
    b2 = fmin(b2, ax * ax + az * az);
  }
  const double best = fmin(sqrt(b2), fabs(r - (even ? g.size[0] : g.size[1])));
  const bool in = r <= g.size[1] || (r <= g.size[0] && even);
  return in ? -best : best;
}

// signed distance of the relaxation region (negative inside it); E: the
// flank table (gear only)
__device__ double ls_phi(const RelaxShape& g, const d2v* E, double x, double y, double z) {
  const double dx = x - g.center[0], dy = y - g.center[1], dz = z - g.center[2];
  double phi;
  switch (g.kind) {
    case SPH_SHAPE_SPHERE: phi = sqrt(dx * dx + dy * dy + dz * dz) - g.size[0]; break;
    case SPH_SHAPE_BOX: {
      const double qx = fabs(dx) - g.size[0], qy = fabs(dy) - g.size[1], qz = fabs(dz) - g.size[2];
      const double ox = fmax(qx, 0.0), oy = fmax(qy, 0.0), oz = fmax(qz, 0.0);
      phi = sqrt(ox * ox + oy * oy + oz * oz) + fmin(fmax(qx, fmax(qy, qz)), 0.0);
      break;
    }
    case SPH_SHAPE_CYLINDER: phi = ls_extrude(sqrt(dx * dx + dz * dz) - g.size[0], dy, g.size[1]); break;
    default: phi = ls_extrude(ls_gear2d(g, E, dx, dz), dy, g.size[2]); break;
  }
  return g.inside ? phi : -phi;
}

// K: relaxation force of eq. 7 on every particle, F_p = -(2/m) V p0 (sum_j V_j
// grad_i W_ij + I_i): the neighbour sum from the rows (as the other sweeps),
// I_i the kernel-gradient integral over the outside of the region (cells of
// edge h/4 over the cube [-2h, 2h]^3, weighted by the outside fraction
// clamp(1/2 + phi/edge, 0, 1)), spread over the 64 lanes of the wavefront for
// each particle that needs it.  Per-block maximum of |F_p|.
template <class P>
__global__ __launch_bounds__(BLOCK) void k_relax_force(const SlotDesc* table, LaunchTab tab, RelaxShape g, int nq) {
  typedef typename P::Real Real;
  typedef typename P::Pos4 Pos4;
  typedef typename P::Real4 Real4;
  __shared__ double red[BLOCK / WAVE];
  __shared__ d2v E[2 * MAX_TEETH];
  __shared__ uint32_t blk_all[BLOCK / WAVE][WAVE];   // active quadrature blocks of a wavefront
  // RQ workgroups per block of BLOCK particles: workgroup `quarter` takes its
  // WAVE particles, every wavefront forms their neighbour sums and wavefront
  // w integrates the exterior of the particles with lane % RQ == w (so the
  // serial per-particle work is spread over RQ times more wavefronts)
  const int vb = xcd_block((int)blockIdx.x, (int)gridDim.x);
  const int quarter = vb % RQ, vblk = vb / RQ;
  int sk = 0;
  for (int s = 1; s < tab.n; ++s)
    if (vblk >= tab.blk0[DOM_FLUID][s]) sk = s;
  const int lb = vblk - tab.blk0[DOM_FLUID][sk];
  const SlotDesc& S = table[tab.slot[sk]];
  if (!live(S)) return;
  ls_flank_table(g, E);
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const int i = lb * BLOCK + quarter * WAVE + lane;
  const bool mine = (lane % RQ) == wv;
  uint32_t* blk = blk_all[wv];
  const bool live_i = i < S.nf;
  const double h = S.h, del = 0.25 * h, vol = S.vol_w, p0 = 1.0;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  double px = 0.0, py = 0.0, pz = 0.0, phx = 0.0;
  bool need = false;
  if (live_i) {
    const GLB Real4* xo = gpc<Real4>(S.xo);
    const Real4 oi = xo[i];
    const uint32_t ci = unpack_index(oi.w);
    const Real inv_h = (Real)(1.0 / h), kF = (Real)S.kF, csr = (Real)S.cs_r;
    Real ax = 0, ay = 0, az = 0;
    const int n = (int)S.nfc[i];
    const GLB uint32_t* R = gpc<uint32_t>(S.nrec) + (int64_t)(i >> 6) * S.kf * WAVE + lane;
    for (int k = 0; k < n; ++k) {
      const uint32_t j = ldnt(R + (int64_t)k * WAVE);
      Real rx, ry, rz;
      pair_vec(oi, ci, xo[j], csr, rx, ry, rz);
      const Real Fk = kernel_F(rx * rx + ry * ry + rz * rz, inv_h, kF);
      ax += Fk * rx;
      ay += Fk * ry;
      az += Fk * rz;
    }
    sx = (double)ax * vol;
    sy = (double)ay * vol;
    sz = (double)az * vol;
    const Pos4 x = gpc<Pos4>(S.xa)[i];
    px = (double)x.x;
    py = (double)x.y;
    pz = (double)x.z;
    phx = ls_phi(g, E, px, py, pz);
    need = phx > -2.0 * h - del;
  }
  // exterior integral, one particle at a time across the wavefront
  double Ix = 0.0, Iy = 0.0, Iz = 0.0;
  uint64_t todo = __ballot(need && mine);
  const double dv = del * del * del, cut = 2.0 * h, inv_h = 1.0 / h, inv_del = 1.0 / del;
  while (todo) {
    const int src = __builtin_ctzll(todo);
    todo &= todo - 1;
    const double qx = __shfl(px, src, WAVE), qy = __shfl(py, src, WAVE), qz = __shfl(pz, src, WAVE);
    const double qphi = __shfl(phx, src, WAVE);
    // phi is a distance (1-Lipschitz): phi(y) <= phi(x) + |x - y|, so a cell
    // with phi(x) + |x - y| <= -edge/2 lies wholly inside.  Skip the prefix of
    // blocks whose every cell is surely that near (block distance plus its
    // half-diagonal below lim, less a margin); the tests below catch the rest.
    int s0 = 0;
    const double lim = -0.5 * del - qphi;
    if (lim > QHALFDIAG * del) {
      const double rb = lim / del - QHALFDIAG;
      const double kl = rb * rb * (1.0 - 1e-9);
      int lo = 0, hi = nq;                       // first entry with key >= kl
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((double)(qcells[mid] >> 12) < kl) lo = mid + 1;
        else hi = mid;
      }
      s0 = lo;
    }
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int s = s0; s < nq; s += WAVE) {
      // one block per lane: its centre's phi bounds all its cells, so a block
      // with phi(centre) + half-diagonal <= -edge/2 has no cell outside, and
      // one with phi(centre) - half-diagonal >= edge/2 has every cell wholly
      // outside (fraction 1, no evaluation of its cells)
      const int q = s + lane;
      uint32_t ent = 0;
      bool act = false, full = false;
      if (q < nq) {
        ent = qcells[q];
        const int A = (int)((ent >> 8) & 15u) - QK / 2, B = (int)((ent >> 4) & 15u) - QK / 2,
                  C = (int)(ent & 15u) - QK / 2;
        const double cx = qx + del * (double)(2 * A + 1), cy = qy + del * (double)(2 * B + 1),
                     cz = qz + del * (double)(2 * C + 1);
        const double ex = qx - cx, ey = qy - cy, ez = qz - cz;
        const double rc = sqrt((ex * ex + ey * ey) + ez * ez);
        if (rc - QHALFDIAG * del < cut && qphi + rc + QHALFDIAG * del > -0.5 * del) {
          const double pc = ls_phi(g, E, cx, cy, cz);
          full = pc - QHALFDIAG * del >= 0.5 * del;
          act = !full && pc + QHALFDIAG * del > -0.5 * del;
        }
      }
      const uint64_t mm = __ballot(act), mf = __ballot(full);
      if (!(mm | mf)) continue;
      // the blocks' codes compacted in lane order, those that need their
      // cells' level set first, then their cells spread over the lanes
      const int nm = __popcll(mm);
      if (act) blk[__builtin_amdgcn_mbcnt_hi((uint32_t)(mm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u))] = ent;
      if (full) blk[nm + __builtin_amdgcn_mbcnt_hi((uint32_t)(mf >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mf, 0u))] = ent;
      relax_lds_sync();
      const int ncm = 8 * nm, ncell = 8 * (nm + __popcll(mf));
      for (int k = lane; k < ncell; k += WAVE) {
        const uint32_t eb = blk[k >> 3];
        const int a = 2 * ((int)((eb >> 8) & 15u) - QK / 2) + (k & 1);
        const int b = 2 * ((int)((eb >> 4) & 15u) - QK / 2) + ((k >> 1) & 1);
        const int c = 2 * ((int)(eb & 15u) - QK / 2) + ((k >> 2) & 1);
        const double yx = qx + del * ((double)a + 0.5), yy = qy + del * ((double)b + 0.5),
                     yz = qz + del * ((double)c + 0.5);
        const double ex = qx - yx, ey = qy - yy, ez = qz - yz;
        const double r2 = (ex * ex + ey * ey) + ez * ez;
        if (!(r2 < cut * cut)) continue;
        const double rr = sqrt(r2);
        if (qphi + rr <= -0.5 * del) continue;
        double f = 1.0;
        if (k < ncm) {
          f = fmin(0.5 + ls_phi(g, E, yx, yy, yz) * inv_del, 1.0);
          if (!(f > 0.0)) continue;
        }
        const double t = 1.0 - 0.5 * rr * inv_h;
        const double F = S.kF * t * t * t;
        const double w = F * (f * dv);
        ax += w * ex;
        ay += w * ey;
        az += w * ez;
      }
      relax_lds_sync();
    }
    ax = wave_sum(ax);
    ay = wave_sum(ay);
    az = wave_sum(az);
    if (lane == src) {
      Ix = ax;
      Iy = ay;
      Iz = az;
    }
  }
  double amag = 0.0;
  if (live_i && mine) {
    const double c = -(2.0 / S.mass) * vol * p0;
    Real4 a;
    a.x = (Real)(c * (sx + Ix));
    a.y = (Real)(c * (sy + Iy));
    a.z = (Real)(c * (sz + Iz));
    a.w = (Real)0;
    gp<Real4>(S.ah)[i] = a;
    const double ax = a.x, ay = a.y, az = a.z;
    amag = sqrt(ax * ax + ay * ay + az * az);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) amag = fmax(amag, __shfl_xor(amag, o, WAVE));
  if (lane == 0) red[threadIdx.x / WAVE] = amag;
  __syncthreads();
  if (threadIdx.x == 0)
    S.glob_part[(size_t)(RELAX_ROW + quarter) * S.nblk[DOM_FLUID] + lb] =
        fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// K: max |F_p| over the blocks, the step of eq. 8, dt = 0.25 sqrt(h / max|F_p|)
__global__ __launch_bounds__(FINAL_BLOCK) void k_relax_max(const SlotDesc* table, LaunchTab tab, int iter) {
  __shared__ double red[FINAL_BLOCK / WAVE];
  SLOT_PROLOGUE(DOM_SLOT);
  (void)lb;
  const int nblk = S.nblk[DOM_FLUID];
  const GLB double* q = gpc<double>(S.glob_part + (size_t)RELAX_ROW * nblk);
  double m = 0.0;
  for (int k = threadIdx.x; k < RQ * nblk; k += FINAL_BLOCK) m = fmax(m, q[k]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, WAVE));
  if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < FINAL_BLOCK / WAVE; ++w) m = fmax(m, red[w]);
  m = fmax(m, red[0]);
  SlotCtl* C = S.ctl;
  C->relax_amax = m;
  C->relax_dt = m > 0.0 ? 0.25 * sqrt(S.h / m) : 0.0;
  if (iter == 0) C->relax_first = m;
  C->relax_bounded = 0;
}

// K: move by eq. 9, x += F_p dt^2 / 2, in FP64 on the anchors; a particle
// that ends with phi > -dp/2 is put back on the level -dp/2 along the unit
// normal (central differences of phi, step 1e-6 h)
template <class P>
__global__ __launch_bounds__(BLOCK) void k_relax_move(const SlotDesc* table, LaunchTab tab, RelaxShape g) {
  typedef typename P::Pos Pos;
  typedef typename P::Pos4 Pos4;
  typedef typename P::Real4 Real4;
  __shared__ d2v E[2 * MAX_TEETH];
  SLOT_PROLOGUE(DOM_FLUID);
  ls_flank_table(g, E);
  __syncthreads();
  const int i = lb * BLOCK + threadIdx.x;
  bool bounded = false;
  if (i < S.nf) {
    const double dt = S.ctl->relax_dt;
    const Real4 a = gpc<Real4>(S.ah)[i];
    GLB Pos4* xa = gp<Pos4>(S.xa);
    Pos4 x4 = xa[i];
    double x[3] = {(double)x4.x, (double)x4.y, (double)x4.z};
    const double ac[3] = {(double)a.x, (double)a.y, (double)a.z};
    for (int k = 0; k < 3; ++k) x[k] += 0.5 * ac[k] * dt * dt;
    const double phi = ls_phi(g, E, x[0], x[1], x[2]);
    if (phi > -0.5 * S.dp) {
      const double eps = 1e-6 * S.h;
      double gr[3];
      for (int k = 0; k < 3; ++k) {
        double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
        xp[k] += eps;
        xm[k] -= eps;
        gr[k] = ls_phi(g, E, xp[0], xp[1], xp[2]) - ls_phi(g, E, xm[0], xm[1], xm[2]);
      }
      const double l = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
      for (int k = 0; k < 3; ++k) x[k] -= (phi + 0.5 * S.dp) * (l > 0.0 ? gr[k] / l : 0.0);
      bounded = true;
    }
    x4.x = (Pos)x[0];
    x4.y = (Pos)x[1];
    x4.z = (Pos)x[2];
    xa[i] = x4;
  }
  const int nb = __syncthreads_count(bounded);
  if (threadIdx.x == 0 && nb > 0) atomicAdd(&S.ctl->relax_bounded, nb);
}

hipError_t launch_relax(int prec, int kid, int iter, const SlotDesc* T, const LaunchTab& L,
                        const RelaxShape& g, hipStream_t st) {
  const int dom = kid == SPH_K_RELAX_MAX ? DOM_SLOT : DOM_FLUID;
  const int nblk = L.blk0[dom][L.n];
  if (nblk <= 0) return hipSuccess;
  const dim3 gr(nblk), b(BLOCK);
  if (kid == SPH_K_RELAX_MAX) {
    hipLaunchKernelGGL(k_relax_max, gr, dim3(FINAL_BLOCK), 0, st, T, L, iter);
    return hipGetLastError();
  }
  if (kid != SPH_K_RELAX_FORCE && kid != SPH_K_RELAX_MOVE) return hipErrorInvalidValue;
  const bool force = kid == SPH_K_RELAX_FORCE;
  const dim3 gq(RQ * nblk);
  int nq = 0;
  if (force) {
    const hipError_t e = qcells_init(&nq);
    if (e != hipSuccess) return e;
  }
  switch (prec) {
    case SPH_PREC_MIXED:
      if (force) hipLaunchKernelGGL(k_relax_force<PMixed>, gq, b, 0, st, T, L, g, nq);
      else hipLaunchKernelGGL(k_relax_move<PMixed>, gr, b, 0, st, T, L, g);
      break;
    case SPH_PREC_FP64:
      if (force) hipLaunchKernelGGL(k_relax_force<PF64>, gq, b, 0, st, T, L, g, nq);
      else hipLaunchKernelGGL(k_relax_move<PF64>, gr, b, 0, st, T, L, g);
      break;
    case SPH_PREC_FP32:
      if (force) hipLaunchKernelGGL(k_relax_force<PF32>, gq, b, 0, st, T, L, g, nq);
      else hipLaunchKernelGGL(k_relax_move<PF32>, gr, b, 0, st, T, L, g);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sphk
