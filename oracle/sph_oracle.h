/*
 * sph_oracle.h -- plain FP64 CPU reference ("oracle") for the gearbox WCSPH
 * hot path of Yu, Wu, Haidn, Hu, "A GPU-Accelerated Fully Coupled
 * Fluid-Solid-Thermal SPH Solver for Industrial Gearboxes" (arXiv 2512.09904).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library and must never be used as a fallback for it.
 *
 * Everything is FP64, compiled with -ffp-contract=off.  Arrays are plain C
 * arrays: vectors are n x 3, row-major (AoS), in the caller's particle order.
 */
#ifndef SPH_ORACLE_H
#define SPH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_OK = 0, ORA_ERR_ARG = 1, ORA_ERR_OOM = 2, ORA_ERR_DOMAIN = 5 };

typedef struct {
  double dp, h_over_dp, rho0, c0, nu, k_f, cp_f;
  double gravity[3];
  double grid_lo[3], grid_hi[3];
  double cfl_ad, cfl_ac;
  double fixed_dt_ad;      /* > 0: use this advection step and fixed_nac sub-steps */
  int32_t fixed_nac;
  int32_t nac_max;         /* cap on acoustic sub-steps per advection step */
  int32_t free_surface;    /* 1: eq. 14 re-initialisation, 0: eq. 15 */
  int32_t eq13_printed;    /* 1: take eq. 13's printed sign (reading study only) */
  int32_t viscous_heating; /* 1: add the dissipation Phi/(rho cp) of eq. 23 to dT/dt */
  int32_t wall_visc;       /* velocity of the dummy particles in eq. 18 (ORA_WALL_VISC_*) */
} ora_params;

/* Dummy-particle velocity v_w in the wall viscous force of eq. 18 (Section
 * 2.5 takes its dummy particles from the generalized wall of Adami et al.
 * 2012, whose no-slip condition extrapolates the fluid velocity into the wall).
 *  SHEPARD (default): v_w = 2 u_w - v~_w, with u_w the body's rigid velocity
 *           at the wall particle and v~_w the kernel-weighted (Shepard) mean
 *           velocity of the fluid within 2h of it; u_w when none is;
 *  RIGID:   v_w = u_w, the body's own velocity (eq. 18 read literally);
 *  PAIR:    v_w = 2 u_w - v_i with the pair's own fluid velocity, i.e.
 *           (v_i - v_w) = 2 (v_i - u_w) (reading study only: unstable at the
 *           viscous step bound of eq. 25). */
enum { ORA_WALL_VISC_SHEPARD = 0, ORA_WALL_VISC_RIGID = 1, ORA_WALL_VISC_PAIR = 2 };

typedef struct { double center[3], axis[3], omega, T, k; } ora_body;

typedef struct {
  double t, dt_ad, dt;
  int32_t n_ac, pad;
  double vmax, mass, kinetic, thermal, heat_step, mass_proxy;
  double diss_step;        /* dt_ad * sum V_i Phi_i (0 without viscous heating) */
} ora_report;

typedef struct { double force[3], torque[3], torque_axis, power, heat_rate; } ora_body_report;

/* Optional per-fluid-particle outputs of ora_step (any pointer may be NULL). */
typedef struct {
  double *a_visc;   /* nf*3 viscous acceleration (frozen for the step) */
  double *dTdt;     /* nf   temperature rate (frozen for the step) */
  double *sumW;     /* nf   kernel sum incl. self, fluid and solid */
  double *S_visc;   /* nf   sum of |viscous pair terms| */
  double *S_T;      /* nf   sum of |heat pair terms| */
  double *a_p;      /* nf*3 pressure acceleration of the last sub-step */
  double *S_p;      /* nf   sum of |pressure pair terms| of the last sub-step */
  double *S_rho;    /* nf   sum of |continuity pair terms| of the last sub-step */
  double *G;        /* nf*9 velocity gradient G[a][b] = d v_a / d x_b (viscous heating only) */
  double *phi;      /* nf   dissipation 2 eta S:S (viscous heating only) */
  double *S_G;      /* nf   sum of |velocity-gradient pair terms| (viscous heating only) */
  double *bscale;   /* nbody*13: per body, the sums of |terms| of its 13 reported parts: viscous
                       force (3) and torque (3), heat flow (1), pressure force (3) and torque (3),
                       the pressure part summed over the sub-steps and divided by n_ac like the
                       report */
} ora_rates;

/* Neighbour sets and the frozen pair geometry of one advection step. */
typedef struct ora_nbr ora_nbr;

/* --- kernel (Wendland C2, support 2h) ------------------------------------ */
double ora_kernel_W(double r, double h);
double ora_kernel_dW(double r, double h);   /* dW/dr */
double ora_kernel_F(double r, double h);    /* (dW/dr)/r, finite at r = 0 */
/* dp^3 * sum over a perfect cubic lattice of W, self included, h = h_over_dp*dp */
double ora_lattice_sum0(double h_over_dp);
/* Lattice kernel sum over the half-space x > 0 seen from a site on x = 0
   (units of dp^3): full-immersion reference of the contact factor, eq. 24. */
double ora_lattice_halfspace(double h_over_dp);

/* --- cells and ordering --------------------------------------------------- */
uint32_t ora_morton3(uint32_t cx, uint32_t cy, uint32_t cz);
int ora_grid_dims(const ora_params* P, int32_t dims[3]);
/* cell coordinates of n points; returns ORA_ERR_DOMAIN if any lies outside */
int ora_cells(const ora_params* P, int64_t n, const double* x, int32_t* cell);
/* order[k] = index of the k-th point in ascending (morton(cell), id) order */
int ora_sort_order(const ora_params* P, int64_t n, const double* x, const uint32_t* id,
                   int64_t* order);

/* --- neighbour search ------------------------------------------------------ */
int ora_nbr_build(const ora_params* P, int64_t nf, const double* xf, int64_t ns,
                  const double* xs, int32_t brute, ora_nbr** out);
int64_t ora_nbr_total(const ora_nbr* nb, int32_t which);   /* 0 fluid, 1 solid */
void ora_nbr_csr(const ora_nbr* nb, int32_t which, int64_t* offsets, int32_t* idx);
void ora_nbr_free(ora_nbr* nb);

/* --- sweeps over frozen neighbour sets ----------------------------------- */
void ora_sum_w(const ora_params* P, const ora_nbr* nb, double* sumW);
/* Contact factor per solid particle (Section 2.7, eq. 24): sum over fluid j
   within 2h of V_j W_wj (V_j = m / rho_j) over ref; zeta[ns]. */
int ora_contact_factor(const ora_params* P, int64_t nf, const double* xf, const double* rho, int64_t ns,
                       const double* xs, double ref, double* zeta);
/* Dummy velocity of every solid particle (ns x 3) under P->wall_visc for the
   fluid velocities v (nf x 3) and the rigid solid velocities vs; also the
   Shepard weight sum_j W_wj (sumW_s, nullable).  PAIR has no per-particle
   value and returns vs. */
void ora_wall_dummy_velocity(const ora_params* P, const ora_nbr* nb, const double* v, const double* vs,
                             double* vd, double* sumW_s);
void ora_viscous(const ora_params* P, const ora_nbr* nb, int32_t nbody, const ora_body* B,
                 const int32_t* body, const double* v, const double* rho, const double* mass,
                 const double* vs, double* a, double* S, double* bforce, double* btorque);
void ora_heat(const ora_params* P, const ora_nbr* nb, int32_t nbody, const ora_body* B,
              const int32_t* body, const double* rho, const double* mass, const double* k,
              const double* cp, const double* T, double* dTdt, double* S, double* bheat);
void ora_momentum(const ora_params* P, const ora_nbr* nb, int32_t nbody, const ora_body* B,
                  const int32_t* body, const double* v, const double* rho, const double* mass,
                  const double* nsv, const double* vs, double* a, double* S, double* bforce,
                  double* btorque);
void ora_continuity(const ora_params* P, const ora_nbr* nb, const double* v,
                    const double* rho, const double* mass, const double* nsv, const double* vs,
                    double* drho, double* S);
/* Velocity gradient G (nf*9, G[a][b] = d v_a / d x_b) from the SPH gradient over
   fluid and wall neighbours, and the viscous dissipation Phi = 2 eta S:S of
   eq. 23 with S = (G + G^T)/2; S (nullable) = sum of |pair terms| per particle. */
void ora_velocity_gradient(const ora_params* P, const ora_nbr* nb, const double* v,
                           const double* rho, const double* mass, const double* vs, double* G,
                           double* S);
void ora_dissipation(const ora_params* P, int64_t nf, const double* G, double* phi);
/* pair forces on i from j: pressure part f[0..2], viscous part f[3..5] */
void ora_pair_force(const ora_params* P, const double* xi, const double* xj, const double* vi,
                    const double* vj, double rhoi, double rhoj, double mi, double mj,
                    double* f);

/* --- bodies, time step, one advection step -------------------------------- */
void ora_body_pose(int32_t nbody, const ora_body* B, int64_t ns, const double* x0,
                   const double* n0, const int32_t* body, double t, double* xs, double* nsv,
                   double* vs);
void ora_timestep(const ora_params* P, int32_t nbody, const ora_body* B, int64_t ns,
                  const double* x0, const int32_t* body, int64_t nf, const double* v,
                  double* dt_ad, double* dt, int32_t* n_ac, double* vmax);
/* the same with the thermal bound dt_T of eq. 26 given (dt_ad <= dt_T) */
void ora_timestep_T(const ora_params* P, int32_t nbody, const ora_body* B, int64_t ns,
                    const double* x0, const int32_t* body, int64_t nf, const double* v, double dt_T,
                    double* dt_ad, double* dt, int32_t* n_ac, double* vmax);
int ora_step(const ora_params* P, int32_t nbody, const ora_body* B, int64_t nf, double* x,
             double* v, double* rho, double* T, double* drho, int64_t ns, const double* x0,
             const double* n0, const int32_t* body, double* t, ora_report* rep,
             ora_body_report* brep, ora_rates* rates);
/* One advection step with per-particle thermal conductivity k_in and specific
   heat cp_in (several fluid materials in eq. 22; either NULL: k_f, cp_f). */
int ora_step_kc(const ora_params* P, int32_t nbody, const ora_body* B, int64_t nf, double* x,
                double* v, double* rho, double* T, double* drho, int64_t ns, const double* x0,
                const double* n0, const int32_t* body, const double* k_in, const double* cp_in,
                double* t, ora_report* rep, ora_body_report* brep, ora_rates* rates);
/* totals of the state: mass, kinetic, thermal, mass proxy, vmax (Neumaier sums);
   the _cp form takes per-particle specific heats (NULL: cp_f) */
void ora_totals(const ora_params* P, int64_t nf, const double* v, const double* rho,
                const double* T, double* out5);
void ora_totals_cp(const ora_params* P, int64_t nf, const double* v, const double* rho,
                   const double* T, const double* cp, double* out5);

/* --- physics-driven particle relaxation (Section 2.2, eq. 5-9) ----------- */
enum { ORA_SHAPE_SPHERE = 1, ORA_SHAPE_BOX = 2, ORA_SHAPE_CYLINDER = 3, ORA_SHAPE_GEAR = 4 };
enum { ORA_RELAX_QK = 8 };   /* exterior integral: (2 K)^3 midpoint cells of edge h/4 */

/* An analytic shape; cylinder and gear have their axis along y.
 * size: sphere (R); box (half extents); cylinder (R, half length);
 * gear (r_tip, r_root, half face width), teeth z, tooth where
 * frac(z theta / 2 pi + 1/4 + phase) < 1/2 with theta = atan2(z - cz, x - cx).
 * inside = 1: the region is the shape; 0: its complement. */
typedef struct {
  int32_t kind, teeth, inside, pad;
  double center[3], size[3], phase;
} ora_shape;

/* signed distance of the region (negative inside it) */
double ora_shape_phi(const ora_shape* s, const double* x);
/* unit gradient of phi by central differences of step eps */
void ora_shape_normal(const ora_shape* s, double eps, const double* x, double* n);
/* int over phi(y) > 0 of grad_x W(x - y) dy (midpoint rule, cells of edge h/4) */
void ora_exterior_integral(const ora_params* P, const ora_shape* s, const double* x, double* I);
/* phi and normals (either nullable) of n points; the exterior integral of n points */
void ora_shape_eval(const ora_shape* s, double eps, int64_t n, const double* x, double* phi, double* nrm);
void ora_exterior_integral_n(const ora_params* P, const ora_shape* s, int64_t n, const double* x, double* I);
/* one relaxation iteration in place; acc (n x 3, nullable) = F_p;
   stats = {max |F_p|, dt, number of particles put back by the confinement} */
int ora_relax_step(const ora_params* P, const ora_shape* s, int64_t n, double* x, double* acc,
                   double* stats);

#ifdef __cplusplus
}
#endif
#endif
