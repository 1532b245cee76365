// sph_internal.h -- shared layout between the host orchestrator and the HIP
// kernels of the WCSPH hot path.  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sph.h"

namespace sphk {

constexpr int BLOCK = 256;          // threads per workgroup (4 wave64)
constexpr int WAVE = 64;            // CDNA wavefront; also the SELL slice height
constexpr int MAX_SLOTS = 32;
constexpr int NB = SPH_MAX_BODIES;
constexpr int NACC = 2;             // distinct bodies one fluid particle may touch
constexpr int NGLOB = 5;            // mass, kinetic, thermal, mass proxy, vmax

enum Dom { DOM_FLUID = 0, DOM_SOLID = 1, DOM_CELL = 2, DOM_SLOT = 3, NDOM = 4 };
enum Flag { F_DOMAIN = 1, F_NONFINITE = 2, F_CAPACITY = 4 };

// Blocks of one launch: the slots it covers and, per domain, the prefix of
// their block counts.  Passed by value (kernel argument segment).
constexpr int32_t TAB_DISS = 1;   // some slot of the launch has viscous heating on
constexpr int32_t TAB_MAT = 2;    // some slot of the launch has several fluid materials
constexpr int NMAT = SPH_MAX_MATERIALS;

struct LaunchTab {
  int32_t n, flags;
  int32_t slot[MAX_SLOTS];
  int32_t blk0[NDOM][MAX_SLOTS + 1];
};

// Device-resident control block of a slot, written only by kernels.
struct SlotCtl {
  double t, dt_ad, dt;
  int64_t step, target, substeps;
  int32_t n_ac;
  uint32_t flags;
  double heat_total, diss_total;
  double relax_amax, relax_dt, relax_first;   // particle relaxation: max |F_p|, step
  int32_t relax_bounded, relax_pad;           // particles put back by the confinement
  double cum[NB][3];     // time integrals: axial torque, energy, heat
  // Neumaier compensation terms of the running totals (cum, heat_total,
  // diss_total): the reported value is the sum plus its compensation
  double cum_c[NB][3];
  double heat_c, diss_c;
  sph_report rep;
  sph_body_report brep[NB];
};

// Everything a kernel needs to know about one slot.  Arrays are in the
// cell-sorted order.  Vectors are stored as 4-wide records (16 B in FP32,
// 32 B in FP64) so that one load or one gather moves a whole record:
//   anchor x (x, y, z, 0)          velocity state (vx, vy, vz, delta-rho)
//   rates (ax, ay, az, dT/dt)       solid lever arm (lx, ly, lz, body index)
//   cell-relative position (ox, oy, oz, packed cell coordinates), frozen at
//   the build: x = lo + c cs_r + o, so r_ij = (o_i - o_j) + (c_i - c_j) cs_r
//   with c_i - c_j in {-1, 0, 1} per axis for every pair
// A neighbour row entry is the neighbour's sorted index (4 B).
struct SlotDesc {
  int32_t nf, ns, ncells, nslices;
  int32_t kf, ks, nbody, nac_bound;
  int32_t dims[3];
  int32_t free_surface, fixed_nac, diss;   // diss: viscous dissipation heating on
  int32_t nblk[NDOM];
  int64_t rowlen_f, rowlen_s;          // nslices * k * 64
  double dp, h, rho0, c0, eta, k_f, cp_f, mass, vol_w, S0, cut2, cs;
  double cs_r;                         // cs rounded to the interaction type (frame of the offsets)
  double zref;                         // full-immersion reference of the contact factor
  double cfl_ad, cfl_ac, fixed_dt_ad, nu;
  double dt_T;                         // thermal bound of eq. 26 over the materials
  double g[3], lo[3];
  double kW, kF;                       // W = kW (1-q/2)^4 (1+2q);  F = kF (1-q/2)^3
  double bc[NB][3], ba[NB][3], bom[NB], bT[NB], bk[NB], btip[NB];
  double mk[NMAT], mcp[NMAT];          // conductivity and specific heat per fluid material
  int32_t nmat;                        // materials (1: every particle takes k_f, cp_f)
  int32_t wall_rigid;                  // eq. 18 with the rigid wall velocity (no Shepard extrapolation)
  SlotCtl* ctl;
  // fluid state (sorted order) and its gather buffers
  void *xa, *drift, *vr, *vrn, *drho, *T, *ah;
  void *td;             // (T, Drho) per sorted particle side by side, 16 B: the fused sweep's gather
  uint32_t *fid;
  double *sumW;
  uint32_t *fcell, *fperm;
  uint64_t *fkey;       // scatter output: (original id << 32) | staged index, per sorted slot
  void *xa2, *vr2, *drho2, *T2;
  uint32_t *fid2;
  uint32_t *mat, *mat2;  // material of each sorted particle and its staging copy (nmat > 1 only)
  // neighbour rows (SELL, slice height 64) of sorted neighbour indices, and
  // the cell-relative positions the sweeps take r_ij from
  uint32_t *nfc, *nsc;
  uint32_t *nrec, *srec;
  uint32_t *rmaj;       // build output: per particle kf fluid then ks solid entries
  void *xo, *so;
  // solids: FP64 reference pose (x, y, z, 0) and normal, body; current pose
  void *x0, *n0;
  int32_t *body;
  uint32_t *sid;
  void *xw, *nw, *vw, *lev;
  void *x0b, *n0b;
  int32_t *bodyb;
  uint32_t *sidb;
  void *xwb, *nwb, *vwb, *levb;
  uint32_t *scell, *sperm;
  double *zeta;         // contact factor per solid particle, original order
  void *vd;             // dummy velocity of eq. 18 per sorted solid particle (vx, vy, vz, dp^3 sum W)
  uint64_t *skey;
  // cells
  uint32_t *rank, *cnt_f, *cnt_s, *start_f, *start_s, *bsum_f, *bsum_s;
  // per fluid-block partials, quantity-major ([quantity][block])
  double *vmax_part;    // per fluid block: max |v| (FP64) for the time step
  double *visc_part;    // [NB * 7]: force(3) torque(3) heat
  double *press_part;   // [NB * 6]: sum over sub-steps of force(3) torque(3)
  double *glob_part;    // [NGLOB + 1]: the globals, then the dissipated power
};

// An analytic shape of the particle relaxation (sph_shape, checked).
struct RelaxShape {
  int32_t kind, teeth, inside, pad;
  double center[3], size[3], phase;
  double zu;            // gear: teeth / (2 pi)
};

// Launch one kernel of the particle relaxation (SPH_K_RELAX_*); iter: the
// iteration index (0 records the first maximum).
hipError_t launch_relax(int prec, int kid, int iter, const SlotDesc* table, const LaunchTab& tab,
                        const RelaxShape& shape, hipStream_t stream);

// Launch one kernel of the step.  prec: SPH_PREC_*; kid: SPH_K_*; sub: the
// acoustic sub-step index (only for the sub-step kernels); which: 0 fluid, 1
// solid (for the kernels launched once per particle set).
hipError_t launch_kernel(int prec, int kid, int which, int sub, const SlotDesc* table,
                         const LaunchTab& tab, hipStream_t stream);
int grid_domain(int kid, int which);

// The contact factor (k_contact) of one slot into zout (caller's order) with,
// when part is given, per-block, per-body partial sums into part (2 x nbody x
// the slot's solid blocks doubles) and, when mean is given, the per-body
// means reduced from them (k_contact_mean).
hipError_t launch_contact(int prec, const SlotDesc* table, const LaunchTab& tab, double* zout, double* part,
                          double* mean, hipStream_t stream);

}  // namespace sphk
