/*
 * sph.h -- C ABI of the MI355X weakly-compressible SPH thermo-fluid hot path.
 *
 * The library advances a lubricant (fluid particles) in a gearbox with
 * prescribed rotating solid bodies, following Yu, Wu, Haidn, Hu, "A
 * GPU-Accelerated Fully Coupled Fluid-Solid-Thermal SPH Solver for Industrial
 * Gearboxes" (arXiv 2512.09904), Section 2:
 *   - Riemann-based continuity and momentum (eq. 10-13),
 *   - density re-initialisation (eq. 14-15),
 *   - dummy-particle walls with a one-sided Riemann problem (eq. 16-19),
 *   - Cleary heat conduction fluid-fluid and fluid-solid (eq. 22),
 *   - dual-criteria time stepping (eq. 25): one neighbour build per advection
 *     step, n_ac acoustic sub-steps on the frozen pair geometry,
 *   - per-body torque, churning power and heat-flow reductions (Section 4).
 * One call of sph_step(s, 1) is one advection step.
 *
 * Conventions.  All functions return an int status (SPH_OK = 0).  No C++
 * exception or abort crosses this boundary; sph_last_error() returns a
 * thread-local message for the last failure.  Host arrays passed in are
 * borrowed for the duration of the call only and copied; vectors are n x 3,
 * row-major (x0 y0 z0 x1 ...), FP64.  Output buffers are owned by the caller.
 * Device memory is obtained only through the sph_allocator given at creation
 * (required: sph_create and sph_pool_create return SPH_ERR_ARG without one;
 * the library never calls hipMalloc itself); all GPU work is enqueued on the
 * HIP stream given at creation (caller-owned; NULL means the legacy default
 * stream, which cannot be graph-captured).  Units are SI; temperatures in K.
 * Gravity points along -z in the workloads but is a parameter.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  SPH_OK = 0,
  SPH_ERR_ARG = 1,        /* invalid argument or parameter */
  SPH_ERR_OOM = 2,        /* the allocator returned NULL */
  SPH_ERR_HIP = 3,        /* a HIP runtime call failed */
  SPH_ERR_STATE = 4,      /* call not valid in the current state (e.g. step before init, faulted) */
  SPH_ERR_DOMAIN = 5,     /* a particle left the cell grid */
  SPH_ERR_NONFINITE = 6,  /* a NaN or Inf appeared in the state or the reductions */
  SPH_ERR_CAPACITY = 7,   /* a neighbour row overflowed, or a particle touched too many bodies */
  SPH_ERR_BUDGET = 8      /* pool admission: no free slot or not enough HBM budget now */
};

/* arithmetic of the interaction sweeps and storage of the state */
enum {
  SPH_PREC_MIXED = 0,  /* FP32 interactions; FP64 position anchors, time, temperature, sums */
  SPH_PREC_FP64 = 1,   /* FP64 everywhere */
  SPH_PREC_FP32 = 2    /* FP32 everywhere: absolute positions, density and temperature */
};

typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* user;
} sph_allocator;

/* Velocity v_w of the dummy particles in the wall viscous force of eq. 18.
 * Section 2.5 takes its dummy particles from the generalized wall boundary of
 * Adami, Hu and Adams (2012), whose no-slip condition extrapolates the fluid
 * velocity into the wall:
 *   SPH_WALL_VISC_SHEPARD (0, default): v_w = 2 u_w - v~_w, u_w the body's
 *     rigid velocity at the wall particle, v~_w the kernel-weighted (Shepard)
 *     mean of the step-start velocity of the fluid particles within 2h of it
 *     (u_w when there are none), summed in FP64 in a fixed order;
 *   SPH_WALL_VISC_RIGID (1): v_w = u_w, eq. 18 read literally (the wall then
 *     slips at the resolutions of the paper).
 * The Riemann wall problem of eq. 16-19 always takes u_w. */
enum { SPH_WALL_VISC_SHEPARD = 0, SPH_WALL_VISC_RIGID = 1 };

/* fluid materials of one solve (thermal properties of eq. 22) */
#define SPH_MAX_MATERIALS 8

/* Problem parameters (Section 2 and Tables 5-6 of the paper). */
typedef struct {
  double dp;            /* particle spacing [m]; fluid mass = rho0 dp^3, solid volume = dp^3 */
  double h_over_dp;     /* smoothing length h / dp, in [1, 2]; kernel support 2h, cell edge 2h */
  double rho0;          /* reference density [kg/m^3] (eq. 2) */
  double c0;            /* artificial sound speed [m/s] (eq. 2) */
  double nu;            /* kinematic viscosity [m^2/s]; eta = rho0 nu */
  double k_f;           /* fluid thermal conductivity [W/(m K)] */
  double cp_f;          /* fluid specific heat [J/(kg K)] */
  double gravity[3];    /* [m/s^2] */
  double grid_lo[3];    /* cell grid lower corner; every particle must stay inside */
  double grid_hi[3];    /* upper corner; at most 1024 cells of edge 2h per axis */
  double cfl_ad;        /* 0.25 (eq. 25) */
  double cfl_ac;        /* 0.6  (eq. 25) */
  double fixed_dt_ad;   /* > 0: fixed advection step (parity runs); 0: eq. 25 */
  int32_t fixed_nac;    /* sub-steps per advection step when fixed_dt_ad > 0 */
  int32_t nac_max;      /* cap on sub-steps; dt_ad is shortened to nac_max dt_ac when hit */
  int32_t free_surface; /* 1: eq. 14 (max with the carried density), 0: eq. 15 */
  int32_t precision;    /* SPH_PREC_* */
  int32_t max_fluid_nbrs; /* neighbour row capacity, 0 = 128; rounded up to a multiple of 16 */
  int32_t max_solid_nbrs; /* solid neighbour row capacity, 0 = 96; rounded up to a multiple of 16 */
  int32_t viscous_heating; /* 1: add the viscous dissipation Phi = 2 eta S:S of eq. 23 (S the strain
                              rate from the SPH velocity gradient over fluid and wall neighbours) to
                              dT/dt as Phi/(rho cp); 0: the paper's model, conduction only */
  int32_t wall_visc;    /* velocity of the dummy particles in the wall viscous force (eq. 18, SPH_WALL_VISC_*);
                           0: the no-slip dummy velocity of the generalized wall Section 2.5 cites */
  int32_t n_materials;  /* 0: one fluid material (k_f, cp_f); 1..SPH_MAX_MATERIALS: the table below,
                           indexed by the per-particle material of sph_set_fluid / sph_pool_admit
                           (eq. 22 with k_i, k_j, cp_i per particle; density and viscosity shared),
                           k_f and cp_f then unused; every k and cp > 0, else SPH_ERR_ARG.  The
                           advection step is also bounded by eq. 26, 0.5 rho0 cp h^2 / k, over the
                           materials */
  int32_t reserved2;    /* must be 0 */
  double mat_k[SPH_MAX_MATERIALS];   /* thermal conductivity of each material [W/(m K)] */
  double mat_cp[SPH_MAX_MATERIALS];  /* specific heat of each material [J/(kg K)] */
} sph_params;

/* A rigid body turning at a prescribed speed about a fixed axis; its solid
 * particles hold the fixed temperature T and conductivity k.  Body 0 is
 * conventionally the static housing (omega = 0).  At most SPH_MAX_BODIES. */
#define SPH_MAX_BODIES 8
typedef struct { double center[3], axis[3], omega, T, k; } sph_body;

/* Global report after the last completed advection step. */
typedef struct {
  double t;             /* simulated time */
  int64_t step;         /* completed advection steps */
  int32_t n_ac;         /* acoustic sub-steps of the last step */
  int32_t flags;        /* latched fault bits: 1 domain, 2 non-finite, 4 capacity (a neighbour row
                           overflowed, or a fluid particle touched more than two bodies) */
  double dt_ad, dt;     /* last advection step and sub-step */
  double vmax;          /* max |v| of the fluid at the end of the step */
  double mass;          /* sum of fluid masses */
  double kinetic;       /* 1/2 sum m |v|^2 */
  double thermal;       /* sum m cp T */
  double heat_step;     /* dt_ad * sum over bodies of the heat flow into the fluid */
  double heat_total;    /* sum of heat_step since init */
  double mass_proxy;    /* sum rho dp^3 (drift of the continuity equation) */
  int64_t substeps;     /* acoustic sub-steps completed since init */
  double diss_step;     /* dt_ad * sum V Phi: heat dissipated in the last step (0 without viscous heating) */
  double diss_total;    /* sum of diss_step since init */
} sph_report;

/* Per-body report: the last step's values (viscous part frozen for the step,
 * pressure part averaged over its sub-steps) and integrals since init. */
typedef struct {
  double force[3];       /* force of the fluid on the body [N] */
  double torque[3];      /* torque about the body centre [N m] */
  double torque_axis;    /* torque component along the body axis */
  double power;          /* -omega * torque_axis: power delivered to the fluid [W] */
  double heat_rate;      /* heat flow from the body into the fluid [W] */
  double torque_axis_int, energy_int, heat_int;   /* time integrals since init */
} sph_body_report;

typedef struct sph_solver sph_solver;
typedef struct sph_pool sph_pool;

const char* sph_error_string(int code);
const char* sph_last_error(void);

/* ---- one solve ----------------------------------------------------------- */
/* Create a solver; nothing is allocated on the device before sph_init.
 * SPH_ERR_ARG for h_over_dp outside [1, 2], non-positive constants, a grid
 * with more than 1024 cells per axis or 2^26 cells in total, or a NULL
 * allocator (or one without alloc or free). */
int sph_create(const sph_params* p, const sph_allocator* a, void* hip_stream, sph_solver** out);
/* Bodies (Section 4, Tables 5-6: each gear turns at a prescribed speed about
 * its shaft and is held at a fixed temperature): n in [1, SPH_MAX_BODIES];
 * axis need not be unit length. */
int sph_set_bodies(sph_solver* s, int32_t n, const sph_body* b);
/* Fluid particles (the lubricant of Section 4, properties of Table 6):
 * positions, velocities, densities, temperatures and material indices
 * (nullable: all 0; each below max(n_materials, 1)); copied at sph_init. */
int sph_set_fluid(sph_solver* s, int64_t n, const double* x, const double* v, const double* rho,
                  const double* T, const int32_t* material);
/* Solid particles at t = 0 in the world frame: positions, unit normals pointing
 * into the fluid, body index of each. */
int sph_set_solid(sph_solver* s, int64_t n, const double* x0, const double* n0,
                  const int32_t* body);
/* Upload, pose bodies at t = 0, sort by cell and build the neighbour rows.
 * SPH_ERR_DOMAIN if a particle lies outside the grid, SPH_ERR_CAPACITY if a row
 * overflows, SPH_ERR_OOM. Synchronises the stream. */
int sph_init(sph_solver* s);
/* Enqueue n advection steps; asynchronous.  Device faults are latched and
 * reported by the next sph_reduce; after a fault, sph_step returns SPH_ERR_STATE. */
int sph_step(sph_solver* s, int32_t n_adv_steps);
/* Synchronise and read the reports (per_body may be NULL; else nbody entries):
 * the observables of Section 4, torque and churning power per shaft and the
 * oil's thermal energy (its mean temperature), with the heat drawn from the
 * bodies.  Returns the latched fault as SPH_ERR_DOMAIN / _NONFINITE /
 * _CAPACITY. */
int sph_reduce(sph_solver* s, sph_report* r, sph_body_report* per_body);
/* Synchronise and read the fluid fields (Section 4: the oil distribution and
 * temperature fields) in the order given to sph_set_fluid.
 * x = anchor + drift; any pointer may be NULL. */
int sph_get_fluid(sph_solver* s, double* x, double* v, double* rho, double* T);
/* Use a captured hipGraph per advection step (default on) or eager launches. */
int sph_set_graph(sph_solver* s, int32_t enable);
/* Per-kernel timing with HIP events on the solver's stream (forces eager launches). */
int sph_set_timing(sph_solver* s, int32_t enable);
/* Durations in ms of the recorded launches of kernel `kernel` (SPH_K_*), oldest
 * first; *count receives the number recorded (may exceed max).  Synchronises. */
int sph_get_timing(sph_solver* s, int32_t kernel, int32_t max, float* ms, int32_t* count);
/* Contact factor (Section 2.7, eq. 24) of every solid particle at the
 * current time t: zeta_w = sum over fluid j with |x_w - x_j| < 2h of
 * V_j W(|x_w - x_j|) (V_j = m / rho_j), divided by the full-immersion
 * reference, the perfect-lattice kernel sum over the wall's outer half-space
 * (0.2133 at h = 1.3 dp): about 1 for a wetted surface particle, 0 in air.
 * zeta: ns doubles in the order of sph_set_solid (may be NULL); body_mean:
 * one double per body, the mean over the body's solid particles (0 for a body
 * without particles; may be NULL).  Runs the cell sort and neighbour build of
 * the current state on the solver's stream (the next step's own build then
 * reproduces them exactly, so stepping is unaffected) and synchronises.
 * SPH_ERR_STATE before sph_init; after a latched fault, that fault's own code
 * (SPH_ERR_DOMAIN / _NONFINITE / _CAPACITY), as sph_reduce returns it. */
int sph_contact_factor(sph_solver* s, double* zeta, double* body_mean);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops that must not call hipMalloc or the host heap): sph_contact_factor
 * with device outputs, no allocation of any kind on success and no
 * synchronisation.  zeta_dev: device buffer of ns doubles, the same values as
 * sph_contact_factor's zeta, bit for bit, in the order of sph_set_solid (may
 * be NULL); body_mean_dev: device buffer of nbody doubles, each body's mean,
 * reduced on the device in a fixed order with compensated sums (equal to
 * sph_contact_factor's host means to about 1e-15 relative; may be NULL).
 * Both are written asynchronously on the solver's stream: the caller
 * synchronises before reading them.  The per-block partial sums live in a
 * static device array of the library (2 MiB, one per GPU, held until the
 * process ends): at most SPH_CONTACT_NOALLOC_MAX_SOLID solid particles, else
 * SPH_ERR_ARG.  Every call on a GPU shares that array, so calls that overlap
 * on one GPU (two streams, two threads) race; calls in stream order do not.
 * SPH_ERR_STATE before sph_init.  A latched fault is not checked here (that
 * would synchronise): the kernels of a faulted solve leave the outputs
 * unwritten and the next sph_reduce returns the fault. */
#define SPH_CONTACT_NOALLOC_MAX_SOLID (4u << 20)
int sph_contact_factor_noalloc(sph_solver* s, double* zeta_dev, double* body_mean_dev);

/* An analytic shape bounding the particle relaxation (Section 2.2, eq. 5):
 * its surface is the zero contour of the signed distance phi, negative inside.
 * Cylinder and gear have their axis along y through the centre.
 *   sphere:   size = (radius, -, -)
 *   box:      size = half extents
 *   cylinder: size = (radius, half length, -)
 *   gear:     size = (tip radius, root radius, half face width), `teeth` teeth
 *             (2 to 512),
 *             tooth where frac(teeth theta / 2 pi + 1/4 + phase) < 1/2 with
 *             theta = atan2(z - cz, x - cx): a root disk with rectangular teeth
 * inside = 1 relaxes within the shape, 0 within its complement. */
enum { SPH_SHAPE_SPHERE = 1, SPH_SHAPE_BOX = 2, SPH_SHAPE_CYLINDER = 3, SPH_SHAPE_GEAR = 4 };
typedef struct {
  int32_t kind, teeth, inside, reserved;
  double center[3], size[3], phase;
} sph_shape;

typedef struct {
  int32_t iterations;     /* iterations done */
  int32_t bounded_last;   /* particles put back by the confinement in the last iteration */
  double amax_first;      /* max |F_p| of the first iteration [m/s^2 per unit p0/rho0] */
  double amax_last;       /* max |F_p| of the last iteration */
  double dt_last;         /* relaxation step of the last iteration (eq. 8) */
} sph_relax_report;

/* Physics-driven particle relaxation (Section 2.2, eq. 6-9) of the solver's
 * fluid particles, which must lie in the region of `shape` (phi < 0), each of
 * volume dp^3 and mass rho0 dp^3, background pressure p0 = 1 (p0 and rho0
 * cancel in the displacement).  Each iteration: cell sort and neighbour build;
 * F_p,i = -(2/m) V p0 (sum_j V grad_i W_ij + I_i) where I_i, the integral of
 * grad W over the outside of the region (phi > 0) on cells of edge h/4
 * weighted by their outside fraction clamp(1/2 + phi/edge, 0, 1), stands in
 * for the neighbours missing beyond the surface; dt = 0.25 sqrt(h / max|F_p|)
 * (eq. 8); x += F_p dt^2 / 2 (eq. 9); a particle ending at phi > -dp/2 is put
 * back on the level -dp/2 along the unit normal (static confinement).  The
 * solver's solid particles take no part.  Only positions change (read them
 * with sph_get_fluid; the density re-initialisation of each build also
 * runs).  Call between steps; synchronises.  SPH_ERR_ARG
 * for a bad shape or iterations < 1, SPH_ERR_DOMAIN if a particle leaves the
 * grid, SPH_ERR_STATE before sph_init; after a latched fault, that fault's own
 * code, as sph_reduce returns it. */
int sph_relax(sph_solver* s, const sph_shape* shape, int32_t iterations, sph_relax_report* report);
/* Raw device state for parity tests (SPH_DUMP_*); bytes must be >= the size
 * reported by sph_dump_size.  Synchronises. */
int sph_dump_size(sph_solver* s, int32_t what, size_t* bytes);
int sph_debug_dump(sph_solver* s, int32_t what, void* buf, size_t bytes);
/* Overwrite one fluid particle's velocity (fault-handling tests; the host
 * makes the state non-finite, no kernel is perturbed). */
int sph_debug_poke_velocity(sph_solver* s, int64_t original_index, const double* v3);
/* enable = 1 (the default): the first acoustic sub-step's opening half update
 * and momentum run inside the viscous/heat sweep; 0: as launches of their
 * own.  Both give the same state bit for bit (the parity tests check it).
 * SPH_ERR_ARG for another value. */
int sph_debug_set_fusion(sph_solver* s, int32_t enable);
int sph_destroy(sph_solver* s);

/* kernels of one advection step (timing ids) */
enum {
  SPH_K_CLEAR = 0, SPH_K_POSE, SPH_K_FOLD, SPH_K_SCAN1, SPH_K_SCAN2, SPH_K_SCAN3, SPH_K_SCATTER,
  SPH_K_CELLSORT, SPH_K_REORDER, SPH_K_BUILD, SPH_K_DT, SPH_K_VISC_HEAT, SPH_K_HALF_A,
  SPH_K_MOMENTUM, SPH_K_CONTINUITY, SPH_K_END, SPH_K_FINAL, SPH_K_SUMW, SPH_K_CONTACT,
  SPH_K_RELAX_FORCE, SPH_K_RELAX_MAX, SPH_K_RELAX_MOVE, SPH_K_WALLVEL, SPH_K_COUNT
};

/* dump selectors; arrays are in the device's cell-sorted order unless noted */
enum {
  SPH_DUMP_FLUID_IDS = 1,   /* uint32[nf]: original index of each sorted fluid particle */
  SPH_DUMP_SOLID_IDS = 2,   /* uint32[ns] */
  SPH_DUMP_FLUID_CELL = 3,  /* uint32[nf]: Morton code of the cell of each sorted particle */
  SPH_DUMP_NBR_COUNT = 4,   /* uint32[2*nf]: fluid counts then solid counts */
  SPH_DUMP_NBR_FLUID = 5,   /* uint32 rows: [nf][kf] sorted index of fluid neighbours (padded) */
  SPH_DUMP_NBR_SOLID = 6,   /* uint32 rows: [nf][ks] sorted index of solid neighbours */
  SPH_DUMP_FLUID_OFFSET = 7,/* double [nf][4]: cell-relative position (3) as stored, packed cell */
  SPH_DUMP_SOLID_OFFSET = 8,/* double [ns][4]: the same for the sorted solids */
  SPH_DUMP_FLUID_STATE = 9, /* double [nf][16]: anchor(3) drift(3) v(3) rho drho T a_visc(3) dTdt */
  SPH_DUMP_SOLID_STATE = 10,/* double [ns][13]: x(3) n(3) v(3) lever(3) body */
  SPH_DUMP_SUMW = 11,       /* double [nf]: kernel sum of the last build */
  SPH_DUMP_SOLID_DUMMY = 12 /* double [ns][4]: dummy velocity of eq. 18 (3), Shepard weight dp^3 sum W */
};

/* ---- serving: many solves stepped together -------------------------------- */
/* Device bytes one solve of this size occupies (what admission charges). */
size_t sph_bytes_required(const sph_params* p, int64_t n_fluid, int64_t n_solid);
/* A pool of up to max_slots (<= 32) concurrent solves sharing one stream and
 * an HBM budget in bytes.  All slots use `precision`.  One pool per host thread. */
int sph_pool_create(size_t hbm_budget, int32_t max_slots, int32_t precision,
                    const sph_allocator* a, void* hip_stream, sph_pool** out);
/* Admit a solve that runs target_steps advection steps.  Returns SPH_ERR_BUDGET
 * when no slot or budget is free now (the caller keeps it queued).  Host arrays
 * as for sph_set_fluid / sph_set_solid; precision in p is ignored. */
int sph_pool_admit(sph_pool* pool, const sph_params* p, int32_t nbody, const sph_body* b,
                   int64_t nf, const double* x, const double* v, const double* rho,
                   const double* T, const int32_t* material, int64_t ns, const double* x0,
                   const double* n0, const int32_t* body, int64_t target_steps, int32_t* slot);
/* Enqueue n advection steps for every active slot that is not held, in
 * batched launches. */
int sph_pool_step(sph_pool* pool, int32_t n_adv_steps);
/* Hold (hold = 1) or resume (hold = 0) an admitted slot.  A held slot is left
 * out of later sph_pool_step calls: its state stays resident and unchanged and
 * it keeps its share of the budget; a resumed slot continues where it stopped,
 * with the same result as if it had never been held.  A scheduler uses this to
 * give the device to a subset of the admitted solves (the shortest remaining
 * ones, say).  A change of the stepped set makes the next sph_pool_step
 * capture a new step graph.  SPH_ERR_ARG for a slot not in use or a hold flag
 * other than 0 or 1. */
int sph_pool_hold(sph_pool* pool, int32_t slot, int32_t hold);
/* Non-blocking: *done = 1 once the slot has finished its target steps (or
 * faulted) and its work has completed on the device; then reports are filled.
 * The return value carries the slot's latched fault, if any.  Until the
 * slot's upload has run on the stream, *done stays 0 and nothing is read. */
int sph_pool_poll(sph_pool* pool, int32_t slot, int32_t* done, sph_report* r,
                  sph_body_report* per_body);
int sph_pool_get_fluid(sph_pool* pool, int32_t slot, double* x, double* v, double* rho,
                       double* T);
/* Free a slot's device memory and return its budget. */
int sph_pool_release(sph_pool* pool, int32_t slot);
/* Bytes currently charged against the budget, and active slot count. */
int sph_pool_usage(sph_pool* pool, size_t* bytes_used, int32_t* active);
int sph_pool_set_graph(sph_pool* pool, int32_t enable);
int sph_pool_destroy(sph_pool* pool);

#ifdef __cplusplus
}
#endif
#endif
