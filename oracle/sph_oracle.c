/*
 * sph_oracle.c -- plain FP64 CPU reference ("oracle") for the WCSPH
 * thermo-fluid hot path of arXiv 2512.09904 (Yu, Wu, Haidn, Hu).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares no
 * code with the HIP library.  Build with -ffp-contract=off so that the
 * cutoff test and the cell index are evaluated exactly as written.
 *
 * Each function states the passage of the paper it follows.  Where the paper
 * is silent the reading adopted is stated at the point of use:
 *  - kernel: Wendland C2 with support 2h (the paper only writes W(r, h));
 *  - neighbours: all particles with squared distance < (2h)^2, evaluated as
 *    (dx*dx + dy*dy) + dz*dz in FP64, self excluded from pair lists;
 *  - Riemann means: arithmetic means for U-bar and P-bar of eq. 12, c = c0;
 *  - eq. 13: the normal component of v* is taken as -U*, so that
 *    (v_i - v*) . e_ij = U* - U_L (the printed sign is a switch);
 *  - wall continuity: mirror state with U*_w = u_w + (P_L - P_R)/(c0 (rho_L + rho_R)),
 *    u_w = -n_w . v_w, rho_R from the equation of state;
 *  - integrator inside the dual-criteria step: position Verlet with
 *    half-step density updates; pair geometry, body pose, viscous and heat
 *    rates frozen for the advection step; temperature by explicit Euler;
 *  - wall viscous force (eq. 18): the dummy particles carry the no-slip
 *    velocity of the generalized wall the paper cites for them,
 *    2 u_w - (Shepard mean of the fluid velocity around w); the literal
 *    rigid velocity is a switch (ora_params.wall_visc);
 *  - torque on a body: sum over wall pairs of (x_w - c_B) x (-f_iw);
 *  - viscous dissipation (eq. 23, optional): S from the SPH velocity
 *    gradient over fluid and wall neighbours;
 *  - thermal step bound (eq. 26): dt_ad <= 0.5 rho0 C_p h^2 / k;
 *  - relaxation (Section 2.2): exterior kernel-gradient integral on cells of
 *    edge h/4 with a linear outside fraction; confinement to phi <= -dp/2.
 *
 * The magnitude of the wall viscous torque is pinned to the Stokes torque
 * between concentric spheres on the wall that does not turn; on a turning
 * wall the pairwise reduction adds the torque it reads for rigid co-rotation
 * of fluid and body (eq. 10 and 18 exchange non-central viscous forces), and
 * that identity is pinned as well.
 */
#include "sph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORA_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Neumaier compensated summation                                             */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } ksum;
static void kadd(ksum* k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
  else k->c += (x - t) + k->s;
  k->s = t;
}
static double kval(const ksum* k) { return k->s + k->c; }

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------------ */
/* Kernel.  The paper writes W(|r_ij|, h) and grad_i W = e_ij dW/dr (eq. 10)  */
/* without naming the function; Wendland C2 in 3D, support 2h:                */
/*   W = a (1 - q/2)^4 (1 + 2q),  a = 21/(16 pi h^3),  q = r/h.               */
/* ------------------------------------------------------------------------ */
double ora_kernel_W(double r, double h) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double a = 21.0 / (16.0 * ORA_PI * h * h * h);
  double s = 1.0 - 0.5 * q;
  return a * s * s * s * s * (1.0 + 2.0 * q);
}

double ora_kernel_dW(double r, double h) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double a = 21.0 / (16.0 * ORA_PI * h * h * h);
  double s = 1.0 - 0.5 * q;
  /* d/dr [ (1-q/2)^4 (1+2q) ] = (1/h) (-5 q)(1-q/2)^3 */
  return -5.0 * a / h * q * s * s * s;
}

double ora_kernel_F(double r, double h) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double a = 21.0 / (16.0 * ORA_PI * h * h * h);
  double s = 1.0 - 0.5 * q;
  return -5.0 * a / (h * h) * s * s * s;
}

/* The reference kernel sum of eq. 14 (sum of W_ij^0 at the initial state) is
 * read as the full-support sum over a perfect cubic lattice, self included. */
double ora_lattice_sum0(double h_over_dp) {
  int R = (int)ceil(2.0 * h_over_dp) + 1;
  double s = 0.0;
  for (int i = -R; i <= R; ++i)
    for (int j = -R; j <= R; ++j)
      for (int k = -R; k <= R; ++k) {
        double r = sqrt((double)(i * i + j * j + k * k));
        s += ora_kernel_W(r, h_over_dp);
      }
  return s;
}

/* Perfect-lattice kernel sum, in units of dp^3, over the sites of the open
   half-space x > 0 as seen from a site on the plane x = 0: the kernel sum of
   a wall particle whose whole outer side is filled with fluid at rho0.  It is
   the full-immersion reference of the contact factor (Section 2.7, eq. 24). */
double ora_lattice_halfspace(double h_over_dp) {
  int R = (int)ceil(2.0 * h_over_dp) + 1;
  double s = 0.0;
  for (int i = 1; i <= R; ++i)
    for (int j = -R; j <= R; ++j)
      for (int k = -R; k <= R; ++k) {
        double r = sqrt((double)(i * i + j * j + k * k));
        s += ora_kernel_W(r, h_over_dp);
      }
  return s;
}

/* ------------------------------------------------------------------------ */
/* Cells (edge 2h) and Morton order.  The paper refreshes neighbour lists      */
/* once per advection step (Section 2.8) but gives no search structure; a    */
/* cell list of edge 2h with Morton-ordered cells is used.                    */
/* ------------------------------------------------------------------------ */
uint32_t ora_morton3(uint32_t cx, uint32_t cy, uint32_t cz) {
  uint32_t key = 0;
  for (int b = 0; b < 10; ++b) {
    key |= ((cx >> b) & 1u) << (3 * b);
    key |= ((cy >> b) & 1u) << (3 * b + 1);
    key |= ((cz >> b) & 1u) << (3 * b + 2);
  }
  return key;
}

static double ora_h(const ora_params* P) { return P->h_over_dp * P->dp; }

int ora_grid_dims(const ora_params* P, int32_t dims[3]) {
  double cs = 2.0 * ora_h(P);
  for (int a = 0; a < 3; ++a) {
    double n = ceil((P->grid_hi[a] - P->grid_lo[a]) / cs);
    if (!(n >= 1.0) || n > 1024.0) return ORA_ERR_ARG;
    dims[a] = (int32_t)n;
  }
  return ORA_OK;
}

int ora_cells(const ora_params* P, int64_t n, const double* x, int32_t* cell) {
  int32_t dims[3];
  if (ora_grid_dims(P, dims)) return ORA_ERR_ARG;
  double cs = 2.0 * ora_h(P);
  int bad = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      double c = floor((x[3 * i + a] - P->grid_lo[a]) / cs);
      if (!(c >= 0.0) || c >= (double)dims[a]) { bad = 1; c = 0.0; }
      cell[3 * i + a] = (int32_t)c;
    }
  return bad ? ORA_ERR_DOMAIN : ORA_OK;
}

typedef struct { uint64_t key; int64_t idx; } keyidx;
static int cmp_keyidx(const void* a, const void* b) {
  uint64_t x = ((const keyidx*)a)->key, y = ((const keyidx*)b)->key;
  return (x > y) - (x < y);
}

int ora_sort_order(const ora_params* P, int64_t n, const double* x, const uint32_t* id,
                   int64_t* order) {
  int32_t* c = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(n > 0 ? n : 1));
  keyidx* k = (keyidx*)malloc(sizeof(keyidx) * (size_t)(n > 0 ? n : 1));
  if (!c || !k) { free(c); free(k); return ORA_ERR_OOM; }
  int rc = ora_cells(P, n, x, c);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t m = ora_morton3((uint32_t)c[3 * i], (uint32_t)c[3 * i + 1], (uint32_t)c[3 * i + 2]);
    k[i].key = (m << 32) | (uint64_t)id[i];
    k[i].idx = i;
  }
  qsort(k, (size_t)n, sizeof(keyidx), cmp_keyidx);
  for (int64_t i = 0; i < n; ++i) order[i] = k[i].idx;
  free(c);
  free(k);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Neighbour sets                                                              */
/* ------------------------------------------------------------------------ */
struct ora_nbr {
  int64_t nf, ns;
  int64_t *off_f, *off_s;
  int32_t *idx_f, *idx_s;
  double *xb, *xsb;   /* positions at the build (frozen geometry) */
  double h;
};

/* squared distance exactly as (dx*dx + dy*dy) + dz*dz */
static double dist2(const double* a, const double* b) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  double s = dx * dx + dy * dy;
  return s + dz * dz;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

typedef struct {
  int64_t n;
  keyidx* k;       /* sorted by morton key (upper bits) */
  int32_t* cell;
} cellset;

static int cellset_make(const ora_params* P, int64_t n, const double* x, cellset* cs) {
  cs->n = n;
  cs->cell = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(n > 0 ? n : 1));
  cs->k = (keyidx*)malloc(sizeof(keyidx) * (size_t)(n > 0 ? n : 1));
  if (!cs->cell || !cs->k) return ORA_ERR_OOM;
  int rc = ora_cells(P, n, x, cs->cell);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t m = ora_morton3((uint32_t)cs->cell[3 * i], (uint32_t)cs->cell[3 * i + 1],
                             (uint32_t)cs->cell[3 * i + 2]);
    cs->k[i].key = (m << 32) | (uint64_t)(uint32_t)i;
    cs->k[i].idx = i;
  }
  qsort(cs->k, (size_t)n, sizeof(keyidx), cmp_keyidx);
  return rc;
}

static void cellset_free(cellset* cs) { free(cs->cell); free(cs->k); }

/* first position in the sorted keys whose morton part is >= m */
static int64_t lower_bound_m(const cellset* cs, uint64_t m) {
  int64_t lo = 0, hi = cs->n;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if ((cs->k[mid].key >> 32) < m) lo = mid + 1; else hi = mid;
  }
  return lo;
}

/* visit the candidates of point x in the 27 cells around cell c */
static int64_t collect(const cellset* cs, const double* xs, const double* x, const int32_t* c,
                       const int32_t* dims, double cut2, int64_t self, int32_t* out) {
  int64_t cnt = 0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int32_t cx = c[0] + dx, cy = c[1] + dy, cz = c[2] + dz;
        if (cx < 0 || cy < 0 || cz < 0 || cx >= dims[0] || cy >= dims[1] || cz >= dims[2]) continue;
        uint64_t m = ora_morton3((uint32_t)cx, (uint32_t)cy, (uint32_t)cz);
        for (int64_t p = lower_bound_m(cs, m); p < cs->n && (cs->k[p].key >> 32) == m; ++p) {
          int64_t j = cs->k[p].idx;
          if (j == self) continue;
          if (dist2(x, xs + 3 * j) < cut2) {
            if (out) out[cnt] = (int32_t)j;
            ++cnt;
          }
        }
      }
  return cnt;
}

static int64_t collect_brute(int64_t n, const double* xs, const double* x, double cut2,
                             int64_t self, int32_t* out) {
  int64_t cnt = 0;
  for (int64_t j = 0; j < n; ++j) {
    if (j == self) continue;
    if (dist2(x, xs + 3 * j) < cut2) {
      if (out) out[cnt] = (int32_t)j;
      ++cnt;
    }
  }
  return cnt;
}

int ora_nbr_build(const ora_params* P, int64_t nf, const double* xf, int64_t ns,
                  const double* xs, int32_t brute, ora_nbr** out) {
  *out = NULL;
  int32_t dims[3];
  if (ora_grid_dims(P, dims)) return ORA_ERR_ARG;
  double h = ora_h(P);
  double two_h = 2.0 * h;
  double cut2 = two_h * two_h;
  ora_nbr* nb = (ora_nbr*)calloc(1, sizeof(ora_nbr));
  if (!nb) return ORA_ERR_OOM;
  nb->nf = nf;
  nb->ns = ns;
  nb->h = h;
  nb->off_f = (int64_t*)calloc((size_t)nf + 1, sizeof(int64_t));
  nb->off_s = (int64_t*)calloc((size_t)nf + 1, sizeof(int64_t));
  nb->xb = (double*)malloc(sizeof(double) * 3 * (size_t)(nf > 0 ? nf : 1));
  nb->xsb = (double*)malloc(sizeof(double) * 3 * (size_t)(ns > 0 ? ns : 1));
  if (!nb->off_f || !nb->off_s || !nb->xb || !nb->xsb) { ora_nbr_free(nb); return ORA_ERR_OOM; }
  memcpy(nb->xb, xf, sizeof(double) * 3 * (size_t)nf);
  if (ns) memcpy(nb->xsb, xs, sizeof(double) * 3 * (size_t)ns);
  cellset cf = {0}, cw = {0};
  int rc = cellset_make(P, nf, xf, &cf);
  int rc2 = cellset_make(P, ns, xs, &cw);
  if (rc == ORA_ERR_OOM || rc2 == ORA_ERR_OOM) { cellset_free(&cf); cellset_free(&cw); ora_nbr_free(nb); return ORA_ERR_OOM; }
  if (rc || rc2) { cellset_free(&cf); cellset_free(&cw); ora_nbr_free(nb); return ORA_ERR_DOMAIN; }
  /* pass 1: counts */
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < nf; ++i) {
    const double* xi = xf + 3 * i;
    if (brute) {
      nb->off_f[i + 1] = collect_brute(nf, xf, xi, cut2, i, NULL);
      nb->off_s[i + 1] = collect_brute(ns, xs, xi, cut2, -1, NULL);
    } else {
      nb->off_f[i + 1] = collect(&cf, xf, xi, cf.cell + 3 * i, dims, cut2, i, NULL);
      nb->off_s[i + 1] = collect(&cw, xs, xi, cf.cell + 3 * i, dims, cut2, -1, NULL);
    }
  }
  for (int64_t i = 0; i < nf; ++i) {
    nb->off_f[i + 1] += nb->off_f[i];
    nb->off_s[i + 1] += nb->off_s[i];
  }
  nb->idx_f = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb->off_f[nf] > 0 ? nb->off_f[nf] : 1));
  nb->idx_s = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb->off_s[nf] > 0 ? nb->off_s[nf] : 1));
  if (!nb->idx_f || !nb->idx_s) { cellset_free(&cf); cellset_free(&cw); ora_nbr_free(nb); return ORA_ERR_OOM; }
  /* pass 2: fill, then sort each list by index */
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < nf; ++i) {
    const double* xi = xf + 3 * i;
    int32_t* of = nb->idx_f + nb->off_f[i];
    int32_t* os = nb->idx_s + nb->off_s[i];
    if (brute) {
      collect_brute(nf, xf, xi, cut2, i, of);
      collect_brute(ns, xs, xi, cut2, -1, os);
    } else {
      collect(&cf, xf, xi, cf.cell + 3 * i, dims, cut2, i, of);
      collect(&cw, xs, xi, cf.cell + 3 * i, dims, cut2, -1, os);
    }
    qsort(of, (size_t)(nb->off_f[i + 1] - nb->off_f[i]), sizeof(int32_t), cmp_i32);
    qsort(os, (size_t)(nb->off_s[i + 1] - nb->off_s[i]), sizeof(int32_t), cmp_i32);
  }
  cellset_free(&cf);
  cellset_free(&cw);
  *out = nb;
  return ORA_OK;
}

int64_t ora_nbr_total(const ora_nbr* nb, int32_t which) {
  return which ? nb->off_s[nb->nf] : nb->off_f[nb->nf];
}

void ora_nbr_csr(const ora_nbr* nb, int32_t which, int64_t* offsets, int32_t* idx) {
  const int64_t* o = which ? nb->off_s : nb->off_f;
  const int32_t* d = which ? nb->idx_s : nb->idx_f;
  memcpy(offsets, o, sizeof(int64_t) * (size_t)(nb->nf + 1));
  memcpy(idx, d, sizeof(int32_t) * (size_t)o[nb->nf]);
}

void ora_nbr_free(ora_nbr* nb) {
  if (!nb) return;
  free(nb->off_f); free(nb->off_s); free(nb->idx_f); free(nb->idx_s);
  free(nb->xb); free(nb->xsb);
  free(nb);
}

/* frozen geometry of pair (i, j): r = x_i - x_j at the build, |r|, F = (dW/dr)/r */
typedef struct { double r[3], rr, F, dW, W; } pgeo;
static void pair_geom(const double* xi, const double* xj, double h, pgeo* g) {
  g->r[0] = xi[0] - xj[0];
  g->r[1] = xi[1] - xj[1];
  g->r[2] = xi[2] - xj[2];
  g->rr = sqrt(dist2(xi, xj));
  g->F = ora_kernel_F(g->rr, h);
  g->dW = ora_kernel_dW(g->rr, h);
  g->W = ora_kernel_W(g->rr, h);
}

/* ------------------------------------------------------------------------ */
/* Density re-initialisation input (Section 2.4, eq. 14-15): sum of W over      */
/* fluid and solid neighbours, self included, unweighted.                    */
/* ------------------------------------------------------------------------ */
void ora_sum_w(const ora_params* P, const ora_nbr* nb, double* sumW) {
  (void)P;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nb->nf; ++i) {
    double s = ora_kernel_W(0.0, nb->h);
    pgeo g;
    for (int64_t p = nb->off_f[i]; p < nb->off_f[i + 1]; ++p) {
      pair_geom(nb->xb + 3 * i, nb->xb + 3 * (int64_t)nb->idx_f[p], nb->h, &g);
      s += g.W;
    }
    for (int64_t p = nb->off_s[i]; p < nb->off_s[i + 1]; ++p) {
      pair_geom(nb->xb + 3 * i, nb->xsb + 3 * (int64_t)nb->idx_s[p], nb->h, &g);
      s += g.W;
    }
    sumW[i] = s;
  }
}

/* per-body accumulation helper: per-particle contributions, then a serial
 * compensated sum in particle order so the result is independent of threads */
typedef struct { double* buf; int64_t nf; int32_t nbody; int32_t width; } bacc;
/* Contact factor of every solid particle (Section 2.7, eq. 24): the sum of
   V_j W(|x_w - x_j|) over the fluid particles j within 2h of solid w, with
   V_j = m / rho_j, divided by the full-immersion reference ref (the same sum
   for the fluid filling the wall's outer half-space at rho0).  The fluid
   particles are taken in index order for each w. */
int ora_contact_factor(const ora_params* P, int64_t nf, const double* xf, const double* rho, int64_t ns,
                       const double* xs, double ref, double* zeta) {
  ora_nbr* nb = NULL;
  int rc = ora_nbr_build(P, nf, xf, ns, xs, 0, &nb);
  if (rc) return rc;
  double h = ora_h(P);
  double m = P->rho0 * P->dp * P->dp * P->dp;
  for (int64_t w = 0; w < ns; ++w) zeta[w] = 0.0;
  for (int64_t i = 0; i < nf; ++i) {
    double Vi = m / rho[i];
    for (int64_t q = nb->off_s[i]; q < nb->off_s[i + 1]; ++q) {
      int32_t w = nb->idx_s[q];
      double r = sqrt(dist2(xf + 3 * i, xs + 3 * (size_t)w));
      zeta[w] += Vi * ora_kernel_W(r, h);
    }
  }
  for (int64_t w = 0; w < ns; ++w) zeta[w] /= ref;
  ora_nbr_free(nb);
  return ORA_OK;
}

static int bacc_init(bacc* a, int64_t nf, int32_t nbody, int32_t width) {
  a->nf = nf; a->nbody = nbody; a->width = width;
  a->buf = (double*)calloc((size_t)(nf > 0 ? nf : 1) * (size_t)(nbody > 0 ? nbody : 1) * (size_t)width, sizeof(double));
  return a->buf ? 0 : -1;
}
static double* bacc_at(bacc* a, int64_t i, int32_t b) { return a->buf + ((size_t)i * (size_t)a->nbody + (size_t)b) * (size_t)a->width; }
static void bacc_reduce(bacc* a, double* out) {
  for (int32_t b = 0; b < a->nbody; ++b)
    for (int32_t w = 0; w < a->width; ++w) {
      ksum k = {0, 0};
      for (int64_t i = 0; i < a->nf; ++i) kadd(&k, bacc_at(a, i, b)[w]);
      out[(size_t)b * (size_t)a->width + (size_t)w] = kval(&k);
    }
  free(a->buf);
}

/* ------------------------------------------------------------------------ */
/* Viscous term: eq. 10 (fluid-fluid, eta_ij = eta for one fluid) and eq. 18   */
/* (fluid-wall, 2 eta_i eta_w/(eta_i + eta_w) = eta with the wall taking the  */
/* fluid's viscosity).  Pair force f_ij = 2 V_i V_j eta (v_i - v_j) F_ij with */
/* F = (dW/dr)/r; a_i = (1/m_i) sum f.  Force on body = -f_iw.                */
/* ------------------------------------------------------------------------ */
static void visc_pair(double Vi, double Vj, double eta, double F, const double* vi,
                      const double* vj, double* f) {
  double c = 2.0 * (Vi * Vj) * eta * F;
  f[0] = c * (vi[0] - vj[0]);
  f[1] = c * (vi[1] - vj[1]);
  f[2] = c * (vi[2] - vj[2]);
}

/* Shepard mean of the fluid velocity around every solid particle w,
 * v~_w = sum_j v_j W_wj / sum_j W_wj over the fluid j within 2h (the frozen
 * build geometry), and the no-slip dummy velocity 2 u_w - v~_w of the
 * generalized wall; a solid particle with no fluid neighbour keeps u_w.  The
 * sums run over the fluid rows in fluid-index order, so the result does not
 * depend on the thread count. */
void ora_wall_dummy_velocity(const ora_params* P, const ora_nbr* nb, const double* v, const double* vs,
                             double* vd, double* sumW_s) {
  if (P->wall_visc != ORA_WALL_VISC_SHEPARD) {
    for (int64_t w = 0; w < nb->ns; ++w) {
      for (int k = 0; k < 3; ++k) vd[3 * w + k] = vs[3 * w + k];
      if (sumW_s) sumW_s[w] = 0.0;
    }
    return;
  }
  double* acc = (double*)calloc((size_t)(nb->ns > 0 ? nb->ns : 1) * 4, sizeof(double));
  if (!acc) abort();
  pgeo g;
  for (int64_t i = 0; i < nb->nf; ++i)
    for (int64_t p = nb->off_s[i]; p < nb->off_s[i + 1]; ++p) {
      int64_t w = nb->idx_s[p];
      pair_geom(nb->xb + 3 * i, nb->xsb + 3 * w, nb->h, &g);
      for (int k = 0; k < 3; ++k) acc[4 * w + k] += v[3 * i + k] * g.W;
      acc[4 * w + 3] += g.W;
    }
  for (int64_t w = 0; w < nb->ns; ++w) {
    for (int k = 0; k < 3; ++k)
      vd[3 * w + k] = acc[4 * w + 3] > 0.0 ? 2.0 * vs[3 * w + k] - acc[4 * w + k] / acc[4 * w + 3]
                                           : vs[3 * w + k];
    if (sumW_s) sumW_s[w] = acc[4 * w + 3];
  }
  free(acc);
}

/* babs (nullable, nbody x 6): per body, the sums over its wall pairs of the
 * absolute values of the force (3) and torque (3) components' terms, the
 * scale against which a differently rounded sum is judged. */
static void viscous_abs(const ora_params* P, const ora_nbr* nb, int32_t nbody, const ora_body* B,
                        const int32_t* body, const double* v, const double* rho, const double* mass,
                        const double* vs, double* a, double* S, double* bforce, double* btorque,
                        double* babs) {
  double eta = P->rho0 * P->nu;
  double Vw = P->dp * P->dp * P->dp;
  bacc acc;
  const int32_t width = babs ? 12 : 6;
  int use_acc = (bforce || btorque || babs) && nbody > 0 && bacc_init(&acc, nb->nf, nbody, width) == 0;
  /* dummy-particle velocity of eq. 18 (reading switch, see ora_params) */
  double* vd = (double*)malloc(sizeof(double) * 3 * (size_t)(nb->ns > 0 ? nb->ns : 1));
  if (!vd) abort();
  ora_wall_dummy_velocity(P, nb, v, vs, vd, NULL);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nb->nf; ++i) {
    double Vi = mass[i] / rho[i];
    double sum[3] = {0, 0, 0}, s_abs = 0.0;
    pgeo g;
    double f[3];
    for (int64_t p = nb->off_f[i]; p < nb->off_f[i + 1]; ++p) {
      int64_t j = nb->idx_f[p];
      pair_geom(nb->xb + 3 * i, nb->xb + 3 * j, nb->h, &g);
      visc_pair(Vi, mass[j] / rho[j], eta, g.F, v + 3 * i, v + 3 * j, f);
      sum[0] += f[0]; sum[1] += f[1]; sum[2] += f[2];
      s_abs += sqrt(dot3(f, f));
    }
    for (int64_t p = nb->off_s[i]; p < nb->off_s[i + 1]; ++p) {
      int64_t w = nb->idx_s[p];
      pair_geom(nb->xb + 3 * i, nb->xsb + 3 * w, nb->h, &g);
      if (P->wall_visc == ORA_WALL_VISC_PAIR) {
        /* v_i - (2 u_w - v_i) = 2 (v_i - u_w) */
        visc_pair(Vi, Vw, eta, g.F, v + 3 * i, vs + 3 * w, f);
        f[0] *= 2.0; f[1] *= 2.0; f[2] *= 2.0;
      } else {
        visc_pair(Vi, Vw, eta, g.F, v + 3 * i, vd + 3 * w, f);
      }
      sum[0] += f[0]; sum[1] += f[1]; sum[2] += f[2];
      s_abs += sqrt(dot3(f, f));
      if (use_acc) {
        int32_t b = body[w];
        double* o = bacc_at(&acc, i, b);
        double fb[3] = {-f[0], -f[1], -f[2]}, l[3], tq[3];
        for (int k = 0; k < 3; ++k) l[k] = nb->xsb[3 * w + k] - B[b].center[k];
        cross3(l, fb, tq);
        for (int k = 0; k < 3; ++k) { o[k] += fb[k]; o[3 + k] += tq[k]; }
        if (babs)
          for (int k = 0; k < 3; ++k) { o[6 + k] += fabs(fb[k]); o[9 + k] += fabs(tq[k]); }
      }
    }
    for (int k = 0; k < 3; ++k) a[3 * i + k] = sum[k] / mass[i];
    if (S) S[i] = s_abs / mass[i];
  }
  free(vd);
  if (use_acc) {
    double* tmp = (double*)malloc(sizeof(double) * (size_t)width * (size_t)nbody);
    if (!tmp) abort();
    bacc_reduce(&acc, tmp);
    for (int32_t b = 0; b < nbody; ++b) {
      for (int k = 0; k < 3; ++k) {
        if (bforce) bforce[3 * b + k] = tmp[width * b + k];
        if (btorque) btorque[3 * b + k] = tmp[width * b + 3 + k];
      }
      if (babs)
        for (int k = 0; k < 6; ++k) babs[6 * b + k] = tmp[width * b + 6 + k];
    }
    free(tmp);
  }
}

void ora_viscous(const ora_params* P, const ora_nbr* nb, int32_t nbody, const ora_body* B,
                 const int32_t* body, const double* v, const double* rho, const double* mass,
                 const double* vs, double* a, double* S, double* bforce, double* btorque) {
  viscous_abs(P, nb, nbody, B, body, v, rho, mass, vs, a, S, bforce, btorque, NULL);
}

/* ------------------------------------------------------------------------ */
/* Heat conduction (Section 2.6, eq. 22):                                        */
/*  dT_i/dt = 1/(rho_i cp_i) [ sum_j V_j K_ij T_ij F_ij + sum_w V_w K_iw T_iw F_iw ] */
/* with K = 4 k_i k_j/(k_i + k_j), T_ij = T_i - T_j, F = (dW/dr)/r.  The wall    */
/* holds the fixed temperature and conductivity of its body.  bheat[b] is the  */
/* heat flow into the fluid from body b: sum m_i cp_i (wall part of dT_i/dt).  */
/* ------------------------------------------------------------------------ */
/* babs (nullable, nbody): per body, the sum of the absolute values of the
 * terms of its heat flow. */
static void heat_abs(const ora_params* P, const ora_nbr* nb, int32_t nbody, const ora_body* B,
                     const int32_t* body, const double* rho, const double* mass, const double* k,
                     const double* cp, const double* T, double* dTdt, double* S, double* bheat,
                     double* babs) {
  double Vw = P->dp * P->dp * P->dp;
  bacc acc;
  const int32_t width = babs ? 2 : 1;
  int use_acc = (bheat || babs) && nbody > 0 && bacc_init(&acc, nb->nf, nbody, width) == 0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nb->nf; ++i) {
    double rc = 1.0 / (rho[i] * cp[i]);
    double sum = 0.0, s_abs = 0.0;
    pgeo g;
    for (int64_t p = nb->off_f[i]; p < nb->off_f[i + 1]; ++p) {
      int64_t j = nb->idx_f[p];
      pair_geom(nb->xb + 3 * i, nb->xb + 3 * j, nb->h, &g);
      double Kij = 4.0 * k[i] * k[j] / (k[i] + k[j]);
      double term = (mass[j] / rho[j]) * Kij * (T[i] - T[j]) * g.F;
      sum += term;
      s_abs += fabs(term);
    }
    for (int64_t p = nb->off_s[i]; p < nb->off_s[i + 1]; ++p) {
      int64_t w = nb->idx_s[p];
      int32_t b = body[w];
      pair_geom(nb->xb + 3 * i, nb->xsb + 3 * w, nb->h, &g);
      double Kiw = 4.0 * k[i] * B[b].k / (k[i] + B[b].k);
      double term = Vw * Kiw * (T[i] - B[b].T) * g.F;
      sum += term;
      s_abs += fabs(term);
      if (use_acc) {
        double* o = bacc_at(&acc, i, b);
        const double q = mass[i] * cp[i] * (rc * term);
        o[0] += q;
        if (babs) o[1] += fabs(q);
      }
    }
    dTdt[i] = rc * sum;
    if (S) S[i] = rc * s_abs;
  }
  if (use_acc) {
    double* tmp = (double*)malloc(sizeof(double) * (size_t)width * (size_t)nbody);
    if (!tmp) abort();
    bacc_reduce(&acc, tmp);
    for (int32_t b = 0; b < nbody; ++b) {
      if (bheat) bheat[b] = tmp[width * b];
      if (babs) babs[b] = tmp[width * b + 1];
    }
    free(tmp);
  }
}

void ora_heat(const ora_params* P, const ora_nbr* nb, int32_t nbody, const ora_body* B,
              const int32_t* body, const double* rho, const double* mass, const double* k,
              const double* cp, const double* T, double* dTdt, double* S, double* bheat) {
  heat_abs(P, nb, nbody, B, body, rho, mass, k, cp, T, dTdt, S, bheat, NULL);
}

/* ------------------------------------------------------------------------ */
/* Viscous dissipation (Section 2.6, eq. 23): Phi = 2 eta S:S with the strain  */
/* rate S = (G + G^T)/2 of the velocity gradient G = grad v.  The paper gives  */
/* no discretisation; G is the SPH gradient of v with the same kernel         */
/* gradient as every other sweep, grad_i W_ij = F_ij r_ij:                     */
/*   G_i[a][b] = sum_j V_j (v_j - v_i)_a F_ij r_ij[b]                          */
/*             + sum_w V_w (v_w - v_i)_a F_iw r_iw[b],                         */
/* walls entering with their rigid-body velocity.  S_G[i] = sum over pairs of  */
/* V |v_j - v_i| |F| |r| bounds the size of every term of every entry.         */
/* ------------------------------------------------------------------------ */
void ora_velocity_gradient(const ora_params* P, const ora_nbr* nb, const double* v,
                           const double* rho, const double* mass, const double* vs, double* G,
                           double* S) {
  double Vw = P->dp * P->dp * P->dp;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nb->nf; ++i) {
    double g[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, s_abs = 0.0;
    pgeo q;
    for (int64_t p = nb->off_f[i]; p < nb->off_f[i + 1]; ++p) {
      int64_t j = nb->idx_f[p];
      pair_geom(nb->xb + 3 * i, nb->xb + 3 * j, nb->h, &q);
      double Vj = mass[j] / rho[j];
      double dv[3] = {v[3 * j] - v[3 * i], v[3 * j + 1] - v[3 * i + 1], v[3 * j + 2] - v[3 * i + 2]};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) g[3 * a + b] += Vj * dv[a] * q.F * q.r[b];
      s_abs += Vj * sqrt(dot3(dv, dv)) * fabs(q.F) * q.rr;
    }
    for (int64_t p = nb->off_s[i]; p < nb->off_s[i + 1]; ++p) {
      int64_t w = nb->idx_s[p];
      pair_geom(nb->xb + 3 * i, nb->xsb + 3 * w, nb->h, &q);
      double dv[3] = {vs[3 * w] - v[3 * i], vs[3 * w + 1] - v[3 * i + 1], vs[3 * w + 2] - v[3 * i + 2]};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) g[3 * a + b] += Vw * dv[a] * q.F * q.r[b];
      s_abs += Vw * sqrt(dot3(dv, dv)) * fabs(q.F) * q.rr;
    }
    for (int k = 0; k < 9; ++k) G[9 * i + k] = g[k];
    if (S) S[i] = s_abs;
  }
}

/* Phi_i = 2 eta S:S, S = (G + G^T)/2, eta = rho0 nu (eq. 23). */
void ora_dissipation(const ora_params* P, int64_t nf, const double* G, double* phi) {
  double eta = P->rho0 * P->nu;
  for (int64_t i = 0; i < nf; ++i) {
    const double* g = G + 9 * i;
    double ss = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double sab = 0.5 * (g[3 * a + b] + g[3 * b + a]);
        ss += sab * sab;
      }
    phi[i] = 2.0 * eta * ss;
  }
}

/* ------------------------------------------------------------------------ */
/* Riemann momentum (Section 2.3, eq. 10-12; walls Section 2.5, eq. 16-19)    */
/* ------------------------------------------------------------------------ */
static double eos_p(const ora_params* P, double rho) { return P->c0 * P->c0 * (rho - P->rho0); }

/* pressure pair force on i from fluid j: -2 V_i V_j p* grad_i W_ij (eq. 10),
 * with the states of eq. 11, p* of eq. 12 (arithmetic P-bar), limiter beta */
static void ff_pressure_pair(const ora_params* P, double Vi, double Vj, double rhoi, double rhoj,
                             const double* vi, const double* vj, const pgeo* g, double* f) {
  if (g->rr == 0.0) { f[0] = f[1] = f[2] = 0.0; return; }
  double e[3] = {g->r[0] / g->rr, g->r[1] / g->rr, g->r[2] / g->rr};
  double pi = eos_p(P, rhoi), pj = eos_p(P, rhoj);
  double UL = -dot3(vi, e), UR = -dot3(vj, e);
  double Pbar = 0.5 * (pi + pj);
  double beta = fmin(3.0 * fmax(UL - UR, 0.0), P->c0);
  double pstar = Pbar + rhoi * rhoj * beta * (UL - UR) / (rhoi + rhoj);
  double c = -2.0 * (Vi * Vj) * pstar * g->dW;
  f[0] = c * e[0];
  f[1] = c * e[1];
  f[2] = c * e[2];
}

/* right state of the one-sided wall problem (eq. 17) and p* of eq. 19 */
typedef struct { double pL, PR, rhoR, pstar; } wallstate;
static void wall_state(const ora_params* P, double rhoi, const pgeo* g, wallstate* s) {
  s->pL = eos_p(P, rhoi);
  double rfw[3] = {-g->r[0], -g->r[1], -g->r[2]};   /* x_w - x_f */
  s->PR = s->pL + rhoi * dot3(P->gravity, rfw);
  s->rhoR = P->rho0 + s->PR / (P->c0 * P->c0);
  s->pstar = (rhoi * s->PR + s->rhoR * s->pL) / (rhoi + s->rhoR);
}

void ora_pair_force(const ora_params* P, const double* xi, const double* xj, const double* vi,
                    const double* vj, double rhoi, double rhoj, double mi, double mj, double* f) {
  pgeo g;
  double h = ora_h(P);
  pair_geom(xi, xj, h, &g);
  if (g.rr >= 2.0 * h) { for (int k = 0; k < 6; ++k) f[k] = 0.0; return; }
  double Vi = mi / rhoi, Vj = mj / rhoj;
  ff_pressure_pair(P, Vi, Vj, rhoi, rhoj, vi, vj, &g, f);
  visc_pair(Vi, Vj, P->rho0 * P->nu, g.F, vi, vj, f + 3);
}

/* babs as for the viscous sweep: sums of |force| and |torque| component terms */
static void momentum_abs(const ora_params* P, const ora_nbr* nb, int32_t nbody, const ora_body* B,
                         const int32_t* body, const double* v, const double* rho, const double* mass,
                         const double* nsv, const double* vs, double* a, double* S, double* bforce,
                         double* btorque, double* babs) {
  (void)nsv; (void)vs;
  double Vw = P->dp * P->dp * P->dp;
  bacc acc;
  const int32_t width = babs ? 12 : 6;
  int use_acc = (bforce || btorque || babs) && nbody > 0 && bacc_init(&acc, nb->nf, nbody, width) == 0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nb->nf; ++i) {
    double Vi = mass[i] / rho[i];
    double sum[3] = {0, 0, 0}, s_abs = 0.0, f[3];
    pgeo g;
    for (int64_t p = nb->off_f[i]; p < nb->off_f[i + 1]; ++p) {
      int64_t j = nb->idx_f[p];
      pair_geom(nb->xb + 3 * i, nb->xb + 3 * j, nb->h, &g);
      ff_pressure_pair(P, Vi, mass[j] / rho[j], rho[i], rho[j], v + 3 * i, v + 3 * j, &g, f);
      sum[0] += f[0]; sum[1] += f[1]; sum[2] += f[2];
      s_abs += sqrt(dot3(f, f));
    }
    for (int64_t p = nb->off_s[i]; p < nb->off_s[i + 1]; ++p) {
      int64_t w = nb->idx_s[p];
      pair_geom(nb->xb + 3 * i, nb->xsb + 3 * w, nb->h, &g);
      if (g.rr == 0.0) continue;
      wallstate ws;
      wall_state(P, rho[i], &g, &ws);
      double e[3] = {g.r[0] / g.rr, g.r[1] / g.rr, g.r[2] / g.rr};
      /* f^{s:p} of eq. 18 with p* of eq. 19 */
      double c = -2.0 * (Vi * Vw) * ws.pstar * g.dW;
      f[0] = c * e[0]; f[1] = c * e[1]; f[2] = c * e[2];
      sum[0] += f[0]; sum[1] += f[1]; sum[2] += f[2];
      s_abs += sqrt(dot3(f, f));
      if (use_acc) {
        int32_t b = body[w];
        double* o = bacc_at(&acc, i, b);
        double fb[3] = {-f[0], -f[1], -f[2]}, l[3], tq[3];
        for (int k = 0; k < 3; ++k) l[k] = nb->xsb[3 * w + k] - B[b].center[k];
        cross3(l, fb, tq);
        for (int k = 0; k < 3; ++k) { o[k] += fb[k]; o[3 + k] += tq[k]; }
        if (babs)
          for (int k = 0; k < 3; ++k) { o[6 + k] += fabs(fb[k]); o[9 + k] += fabs(tq[k]); }
      }
    }
    for (int k = 0; k < 3; ++k) a[3 * i + k] = sum[k] / mass[i];
    if (S) S[i] = s_abs / mass[i];
  }
  if (use_acc) {
    double* tmp = (double*)malloc(sizeof(double) * (size_t)width * (size_t)nbody);
    if (!tmp) abort();
    bacc_reduce(&acc, tmp);
    for (int32_t b = 0; b < nbody; ++b) {
      for (int k = 0; k < 3; ++k) {
        if (bforce) bforce[3 * b + k] = tmp[width * b + k];
        if (btorque) btorque[3 * b + k] = tmp[width * b + 3 + k];
      }
      if (babs)
        for (int k = 0; k < 6; ++k) babs[6 * b + k] = tmp[width * b + 6 + k];
    }
    free(tmp);
  }
}

void ora_momentum(const ora_params* P, const ora_nbr* nb, int32_t nbody, const ora_body* B,
                  const int32_t* body, const double* v, const double* rho, const double* mass,
                  const double* nsv, const double* vs, double* a, double* S, double* bforce,
                  double* btorque) {
  momentum_abs(P, nb, nbody, B, body, v, rho, mass, nsv, vs, a, S, bforce, btorque, NULL);
}

/* ------------------------------------------------------------------------ */
/* Riemann continuity (eq. 10 first line, eq. 11-13):                           */
/*   drho_i/dt = 2 rho_i sum_j V_j (v_i - v*) . grad_i W_ij                      */
/* with (v_i - v*) . e_ij = U* - U_L (eq. 13 read with the normal component of  */
/* v* equal to -U*).  Walls: mirror state, (v_i - v*) = (U*_w - U_L) n_w.       */
/* ------------------------------------------------------------------------ */
void ora_continuity(const ora_params* P, const ora_nbr* nb, const double* v,
                    const double* rho, const double* mass, const double* nsv, const double* vs,
                    double* drho, double* S) {
  double Vw = P->dp * P->dp * P->dp;
  double c0 = P->c0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nb->nf; ++i) {
    double sum = 0.0, s_abs = 0.0;
    pgeo g;
    const double* vi = v + 3 * i;
    double pi = eos_p(P, rho[i]);
    for (int64_t p = nb->off_f[i]; p < nb->off_f[i + 1]; ++p) {
      int64_t j = nb->idx_f[p];
      pair_geom(nb->xb + 3 * i, nb->xb + 3 * j, nb->h, &g);
      if (g.rr == 0.0) continue;
      double e[3] = {g.r[0] / g.rr, g.r[1] / g.rr, g.r[2] / g.rr};
      double pj = eos_p(P, rho[j]);
      double UL = -dot3(vi, e), UR = -dot3(v + 3 * j, e);
      double Ubar = 0.5 * (UL + UR);
      double Ustar = Ubar + (pi - pj) / (c0 * (rho[i] + rho[j]));
      double dvn;
      if (P->eq13_printed) {
        double rU = (rho[i] * UL + rho[j] * UR) / (rho[i] + rho[j]);
        dvn = 2.0 * rU - UL - Ustar;
      } else {
        dvn = Ustar - UL;
      }
      double term = 2.0 * rho[i] * (mass[j] / rho[j]) * dvn * g.dW;
      sum += term;
      s_abs += fabs(term);
    }
    for (int64_t p = nb->off_s[i]; p < nb->off_s[i + 1]; ++p) {
      int64_t w = nb->idx_s[p];
      pair_geom(nb->xb + 3 * i, nb->xsb + 3 * w, nb->h, &g);
      if (g.rr == 0.0) continue;
      const double* nw = nsv + 3 * w;
      double e[3] = {g.r[0] / g.rr, g.r[1] / g.rr, g.r[2] / g.rr};
      wallstate ws;
      wall_state(P, rho[i], &g, &ws);
      double UL = -dot3(nw, vi);
      double uw = -dot3(nw, vs + 3 * w);
      double Ustar = uw + (ws.pL - ws.PR) / (c0 * (rho[i] + ws.rhoR));
      double term = 2.0 * rho[i] * Vw * (Ustar - UL) * dot3(nw, e) * g.dW;
      sum += term;
      s_abs += fabs(term);
    }
    drho[i] = sum;
    if (S) S[i] = s_abs;
  }
}

/* ------------------------------------------------------------------------ */
/* Prescribed rigid rotation of the gears (Section 4: gears turn at fixed      */
/* speed and uniform temperature).  Angle omega*t from the FP64 time, never     */
/* accumulated; Rodrigues' rotation about the body's unit axis.                */
/* ------------------------------------------------------------------------ */
static void rotate(const double* a, double c, double s, const double* u, double* out) {
  double axu[3];
  cross3(a, u, axu);
  double au = dot3(a, u);
  for (int k = 0; k < 3; ++k) out[k] = u[k] * c + axu[k] * s + a[k] * au * (1.0 - c);
}

static void unit_axis(const ora_body* b, double* a) {
  double n = sqrt(dot3(b->axis, b->axis));
  a[0] = b->axis[0] / n; a[1] = b->axis[1] / n; a[2] = b->axis[2] / n;
}

void ora_body_pose(int32_t nbody, const ora_body* B, int64_t ns, const double* x0,
                   const double* n0, const int32_t* body, double t, double* xs, double* nsv,
                   double* vs) {
  (void)nbody;
  for (int64_t w = 0; w < ns; ++w) {
    const ora_body* b = &B[body[w]];
    double a[3], u[3], ru[3];
    unit_axis(b, a);
    double th = b->omega * t;
    double c = cos(th), s = sin(th);
    for (int k = 0; k < 3; ++k) u[k] = x0[3 * w + k] - b->center[k];
    rotate(a, c, s, u, ru);
    for (int k = 0; k < 3; ++k) xs[3 * w + k] = b->center[k] + ru[k];
    rotate(a, c, s, n0 + 3 * w, nsv + 3 * w);
    double wa[3] = {b->omega * a[0], b->omega * a[1], b->omega * a[2]};
    cross3(wa, ru, vs + 3 * w);
  }
}

/* ------------------------------------------------------------------------ */
/* Dual-criteria time step (Section 2.8, eq. 25): |v|max includes the bodies'  */
/* tip speeds; n_ac = ceil(dt_ad/dt_ac) sub-steps of dt = dt_ad/n_ac; n_ac is   */
/* capped at nac_max by shortening dt_ad.                                       */
/* ------------------------------------------------------------------------ */
void ora_timestep(const ora_params* P, int32_t nbody, const ora_body* B, int64_t ns,
                  const double* x0, const int32_t* body, int64_t nf, const double* v,
                  double* dt_ad, double* dt, int32_t* n_ac, double* vmax) {
  double h = ora_h(P);
  ora_timestep_T(P, nbody, B, ns, x0, body, nf, v, 0.5 * P->rho0 * P->cp_f * h * h / P->k_f, dt_ad, dt,
                 n_ac, vmax);
}

/* eq. 25 with the thermal bound of eq. 26, dt_T = 0.5 rho C_p h^2 / k (rho
   read as rho0), applied as dt_ad <= dt_T before the sub-steps are counted */
void ora_timestep_T(const ora_params* P, int32_t nbody, const ora_body* B, int64_t ns,
                    const double* x0, const int32_t* body, int64_t nf, const double* v, double dt_T,
                    double* dt_ad, double* dt, int32_t* n_ac, double* vmax) {
  double h = ora_h(P);
  double vm = 0.0;
  for (int64_t i = 0; i < nf; ++i) {
    double s = sqrt(dot3(v + 3 * i, v + 3 * i));
    if (s > vm) vm = s;
  }
  for (int64_t w = 0; w < ns; ++w) {
    const ora_body* b = &B[body[w]];
    if (b->omega == 0.0) continue;
    double a[3], u[3];
    unit_axis(b, a);
    for (int k = 0; k < 3; ++k) u[k] = x0[3 * w + k] - b->center[k];
    double au = dot3(a, u);
    double d[3] = {u[0] - au * a[0], u[1] - au * a[1], u[2] - au * a[2]};
    double s = fabs(b->omega) * sqrt(dot3(d, d));
    if (s > vm) vm = s;
  }
  (void)nbody;
  *vmax = vm;
  if (P->fixed_dt_ad > 0.0) {
    *dt_ad = P->fixed_dt_ad;
    *n_ac = P->fixed_nac > 0 ? P->fixed_nac : 1;
    *dt = *dt_ad / (double)(*n_ac);
    return;
  }
  double visc = h * h / P->nu;
  double adv = vm > 0.0 ? h / vm : visc;
  double tad = P->cfl_ad * (adv < visc ? adv : visc);
  if (dt_T < tad) tad = dt_T;
  double tac = P->cfl_ac * h / (P->c0 + vm);
  double n = ceil(tad / tac);
  if (n < 1.0) n = 1.0;
  if (n > (double)P->nac_max) { n = (double)P->nac_max; tad = n * tac; }
  *dt_ad = tad;
  *n_ac = (int32_t)n;
  *dt = tad / n;
}

void ora_totals(const ora_params* P, int64_t nf, const double* v, const double* rho,
                const double* T, double* out5) {
  ora_totals_cp(P, nf, v, rho, T, NULL, out5);
}

void ora_totals_cp(const ora_params* P, int64_t nf, const double* v, const double* rho,
                   const double* T, const double* cp, double* out5) {
  double m = P->rho0 * P->dp * P->dp * P->dp;
  ksum km = {0, 0}, ke = {0, 0}, kt = {0, 0}, kp = {0, 0};
  double vm = 0.0;
  for (int64_t i = 0; i < nf; ++i) {
    double v2 = dot3(v + 3 * i, v + 3 * i);
    kadd(&km, m);
    kadd(&ke, 0.5 * m * v2);
    kadd(&kt, m * (cp ? cp[i] : P->cp_f) * T[i]);
    kadd(&kp, rho[i] * P->dp * P->dp * P->dp);
    if (sqrt(v2) > vm) vm = sqrt(v2);
  }
  out5[0] = kval(&km); out5[1] = kval(&ke); out5[2] = kval(&kt); out5[3] = kval(&kp); out5[4] = vm;
}

/* ------------------------------------------------------------------------ */
/* One advection step.                                                           */
/* ------------------------------------------------------------------------ */
int ora_step(const ora_params* P, int32_t nbody, const ora_body* B, int64_t nf, double* x,
             double* v, double* rho, double* T, double* drho, int64_t ns, const double* x0,
             const double* n0, const int32_t* body, double* t, ora_report* rep,
             ora_body_report* brep, ora_rates* rates) {
  return ora_step_kc(P, nbody, B, nf, x, v, rho, T, drho, ns, x0, n0, body, NULL, NULL, t, rep, brep, rates);
}

int ora_step_kc(const ora_params* P, int32_t nbody, const ora_body* B, int64_t nf, double* x,
                double* v, double* rho, double* T, double* drho, int64_t ns, const double* x0,
                const double* n0, const int32_t* body, const double* k_in, const double* cp_in,
                double* t, ora_report* rep, ora_body_report* brep, ora_rates* rates) {
  int rc = ORA_OK;
  double dp3 = P->dp * P->dp * P->dp;
  double m0 = P->rho0 * dp3;
  size_t nfz = (size_t)(nf > 0 ? nf : 1), nsz = (size_t)(ns > 0 ? ns : 1);
  double *xs = malloc(sizeof(double) * 3 * nsz), *nsv = malloc(sizeof(double) * 3 * nsz),
         *vs = malloc(sizeof(double) * 3 * nsz);
  double *mass = malloc(sizeof(double) * nfz), *kf = malloc(sizeof(double) * nfz),
         *cpf = malloc(sizeof(double) * nfz), *sumW = malloc(sizeof(double) * nfz),
         *av = malloc(sizeof(double) * 3 * nfz), *ap = malloc(sizeof(double) * 3 * nfz),
         *dTdt = malloc(sizeof(double) * nfz);
  double *G = NULL, *phi = NULL, *SG = NULL;
  double* bq = calloc((size_t)(nbody > 0 ? nbody : 1), sizeof(double));
  double* bFv = calloc(3 * (size_t)(nbody > 0 ? nbody : 1), sizeof(double));
  double* bTv = calloc(3 * (size_t)(nbody > 0 ? nbody : 1), sizeof(double));
  double* bFp = calloc(3 * (size_t)(nbody > 0 ? nbody : 1), sizeof(double));
  double* bTp = calloc(3 * (size_t)(nbody > 0 ? nbody : 1), sizeof(double));
  ksum* kFp = calloc(6 * (size_t)(nbody > 0 ? nbody : 1), sizeof(ksum));
  /* scales of the body quantities (rates->bscale): |terms| of the viscous part
     (6), the heat flow (1) and the pressure part summed over the sub-steps (6) */
  double* babs = calloc(13 * (size_t)(nbody > 0 ? nbody : 1), sizeof(double));
  double* bsub = calloc(6 * (size_t)(nbody > 0 ? nbody : 1), sizeof(double));
  const int want_scale = rates && rates->bscale && nbody > 0;
  ora_nbr* nb = NULL;
  if (!xs || !nsv || !vs || !mass || !kf || !cpf || !sumW || !av || !ap || !dTdt || !bq || !bFv ||
      !bTv || !bFp || !bTp || !kFp || !babs || !bsub) { rc = ORA_ERR_OOM; goto done; }
  if (P->viscous_heating) {
    G = malloc(sizeof(double) * 9 * nfz);
    phi = malloc(sizeof(double) * nfz);
    SG = malloc(sizeof(double) * nfz);
    if (!G || !phi || !SG) { rc = ORA_ERR_OOM; goto done; }
  }
  for (int64_t i = 0; i < nf; ++i) {
    mass[i] = m0;
    kf[i] = k_in ? k_in[i] : P->k_f;
    cpf[i] = cp_in ? cp_in[i] : P->cp_f;
  }

  /* 1. bodies at t_n */
  ora_body_pose(nbody, B, ns, x0, n0, body, *t, xs, nsv, vs);
  /* 2-3. cells, neighbour sets, frozen geometry (Section 2.8) */
  rc = ora_nbr_build(P, nf, x, ns, xs, 0, &nb);
  if (rc) goto done;
  /* 4. density re-initialisation (Section 2.4) */
  ora_sum_w(P, nb, sumW);
  {
    double S0 = ora_lattice_sum0(P->h_over_dp);
    for (int64_t i = 0; i < nf; ++i) {
      double r0 = P->rho0 * (dp3 * sumW[i]) / S0;
      rho[i] = P->free_surface ? fmax(rho[i], r0) : r0;
    }
  }
  /* 5. time step (Section 2.8) */
  double dt_ad, dt, vmax0;
  int32_t n_ac;
  double dtT = INFINITY;
  for (int64_t i = 0; i < nf; ++i) {
    double hh = ora_h(P);
    double d = 0.5 * P->rho0 * cpf[i] * hh * hh / kf[i];
    if (d < dtT) dtT = d;
  }
  ora_timestep_T(P, nbody, B, ns, x0, body, nf, v, dtT, &dt_ad, &dt, &n_ac, &vmax0);
  /* 6. viscous and heat rates, frozen for the step */
  {
    double* vabs = want_scale ? malloc(sizeof(double) * 6 * (size_t)nbody) : NULL;
    double* habs = want_scale ? malloc(sizeof(double) * (size_t)nbody) : NULL;
    if (want_scale && (!vabs || !habs)) { free(vabs); free(habs); rc = ORA_ERR_OOM; goto done; }
    viscous_abs(P, nb, nbody, B, body, v, rho, mass, vs, av, rates ? rates->S_visc : NULL, bFv, bTv, vabs);
    heat_abs(P, nb, nbody, B, body, rho, mass, kf, cpf, T, dTdt, rates ? rates->S_T : NULL, bq, habs);
    if (want_scale)
      for (int32_t b = 0; b < nbody; ++b) {
        for (int k = 0; k < 6; ++k) babs[13 * b + k] = vabs[6 * b + k];
        babs[13 * b + 6] = habs[b];
      }
    free(vabs);
    free(habs);
  }
  /* viscous dissipation heating, eq. 23 (off in the paper's model) */
  ksum kd = {0, 0};
  if (P->viscous_heating) {
    ora_velocity_gradient(P, nb, v, rho, mass, vs, G, SG);
    ora_dissipation(P, nf, G, phi);
    for (int64_t i = 0; i < nf; ++i) {
      dTdt[i] += phi[i] / (rho[i] * cpf[i]);
      kadd(&kd, (mass[i] / rho[i]) * phi[i]);
    }
  }
  /* 7. acoustic sub-steps */
  for (int32_t s = 0; s < n_ac; ++s) {
    for (int64_t i = 0; i < nf; ++i) {
      rho[i] += 0.5 * dt * drho[i];
      for (int k = 0; k < 3; ++k) x[3 * i + k] += 0.5 * dt * v[3 * i + k];
    }
    momentum_abs(P, nb, nbody, B, body, v, rho, mass, nsv, vs, ap, rates ? rates->S_p : NULL, bFp, bTp,
                 want_scale ? bsub : NULL);
    for (int32_t b = 0; b < nbody; ++b)
      for (int k = 0; k < 3; ++k) { kadd(&kFp[6 * b + k], bFp[3 * b + k]); kadd(&kFp[6 * b + 3 + k], bTp[3 * b + k]); }
    if (want_scale)
      for (int32_t b = 0; b < nbody; ++b)
        for (int k = 0; k < 6; ++k) babs[13 * b + 7 + k] += bsub[6 * b + k];
    for (int64_t i = 0; i < nf; ++i)
      for (int k = 0; k < 3; ++k) {
        v[3 * i + k] += dt * (ap[3 * i + k] + av[3 * i + k] + P->gravity[k]);
        x[3 * i + k] += 0.5 * dt * v[3 * i + k];
      }
    ora_continuity(P, nb, v, rho, mass, nsv, vs, drho, rates ? rates->S_rho : NULL);
    for (int64_t i = 0; i < nf; ++i) rho[i] += 0.5 * dt * drho[i];
  }
  /* 8. temperature, explicit Euler over the advection step */
  for (int64_t i = 0; i < nf; ++i) T[i] += dt_ad * dTdt[i];
  *t += dt_ad;
  /* 9. reports */
  if (brep) {
    for (int32_t b = 0; b < nbody; ++b) {
      double a[3];
      unit_axis(&B[b], a);
      for (int k = 0; k < 3; ++k) {
        brep[b].force[k] = bFv[3 * b + k] + kval(&kFp[6 * b + k]) / (double)n_ac;
        brep[b].torque[k] = bTv[3 * b + k] + kval(&kFp[6 * b + 3 + k]) / (double)n_ac;
      }
      brep[b].torque_axis = dot3(a, brep[b].torque);
      brep[b].power = -B[b].omega * brep[b].torque_axis;
      brep[b].heat_rate = bq[b];
    }
  }
  if (rep) {
    double tot[5];
    ora_totals_cp(P, nf, v, rho, T, cpf, tot);
    ksum kq = {0, 0};
    for (int32_t b = 0; b < nbody; ++b) kadd(&kq, bq[b]);
    rep->t = *t; rep->dt_ad = dt_ad; rep->dt = dt; rep->n_ac = n_ac; rep->pad = 0;
    rep->vmax = tot[4]; rep->mass = tot[0]; rep->kinetic = tot[1]; rep->thermal = tot[2];
    rep->mass_proxy = tot[3];
    rep->heat_step = dt_ad * kval(&kq);
    rep->diss_step = dt_ad * kval(&kd);
  }
  if (rates) {
    if (rates->a_visc) memcpy(rates->a_visc, av, sizeof(double) * 3 * (size_t)nf);
    if (rates->dTdt) memcpy(rates->dTdt, dTdt, sizeof(double) * (size_t)nf);
    if (rates->sumW) memcpy(rates->sumW, sumW, sizeof(double) * (size_t)nf);
    if (rates->a_p) memcpy(rates->a_p, ap, sizeof(double) * 3 * (size_t)nf);
    if (want_scale)
      for (int32_t b = 0; b < nbody; ++b)
        for (int k = 0; k < 13; ++k) rates->bscale[13 * b + k] = k < 7 ? babs[13 * b + k] : babs[13 * b + k] / (double)n_ac;
    if (P->viscous_heating) {
      if (rates->G) memcpy(rates->G, G, sizeof(double) * 9 * (size_t)nf);
      if (rates->phi) memcpy(rates->phi, phi, sizeof(double) * (size_t)nf);
      if (rates->S_G) memcpy(rates->S_G, SG, sizeof(double) * (size_t)nf);
    }
  }
done:
  ora_nbr_free(nb);
  free(xs); free(nsv); free(vs); free(mass); free(kf); free(cpf); free(sumW); free(av); free(ap);
  free(dTdt); free(bq); free(bFv); free(bTv); free(bFp); free(bTp); free(kFp); free(babs); free(bsub);
  free(G); free(phi); free(SG);
  return rc;
}

/* ======================================================================== */
/* Physics-driven particle relaxation (Section 2.2, eq. 5-9)                  */
/* ======================================================================== */

/* Level sets of the analytic shapes (eq. 5: the surface is the zero contour, */
/* negative inside).  Every function returns the exact signed distance.       */
static double len2(double a, double b) { return sqrt(a * a + b * b); }

/* extrusion along y of a cross-section with signed distance d2 over the slab */
/* |y| <= half: exact distance of the intersection of the prism and the slab  */
static double extrude(double d2, double y, double half) {
  double dy = fabs(y) - half;
  double ox = d2 > 0.0 ? d2 : 0.0, oy = dy > 0.0 ? dy : 0.0;
  double in = d2 > dy ? d2 : dy;
  return len2(ox, oy) + (in < 0.0 ? in : 0.0);
}

/* distance from (px, pz) to the arc of radius R between tooth coordinates   */
/* u0 < u1 (angle theta = 2 pi (u - 1/4 - phase) / z)                         */
static double arc_dist(double px, double pz, double r, double u, double R, double u0, double u1, int z,
                       double phase) {
  if (u >= u0 && u <= u1) return fabs(r - R);
  double best = INFINITY;
  for (int e = 0; e < 2; ++e) {
    double th = 2.0 * ORA_PI * ((e ? u1 : u0) - 0.25 - phase) / (double)z;
    double d = len2(px - R * cos(th), pz - R * sin(th));
    if (d < best) best = d;
  }
  return best;
}

/* distance from (px, pz) to the radial flank at tooth coordinate u, r in [r0, r1] */
static double flank_dist(double px, double pz, double u, double r0, double r1, int z, double phase) {
  double th = 2.0 * ORA_PI * (u - 0.25 - phase) / (double)z;
  double ex = cos(th), ez = sin(th);
  double t = px * ex + pz * ez;
  if (t < r0) t = r0;
  if (t > r1) t = r1;
  return len2(px - t * ex, pz - t * ez);
}

/* Gear cross-section (axis y): root disk r <= r_root plus teeth up to r_tip   */
/* where the tooth coordinate u = z theta / 2 pi + 1/4 + phase has frac(u) <  */
/* 1/2.  Its boundary: tip arcs over teeth, root arcs over gaps, radial flanks */
/* at the half-integers of u.  The nearest boundary point lies on the pieces  */
/* of the half-pitch holding the point or of its two neighbours.              */
static double gear_section(double px, double pz, int z, double r_tip, double r_root, double phase) {
  double r = len2(px, pz);
  double u = (double)z * atan2(pz, px) / (2.0 * ORA_PI) + 0.25 + phase;
  double k = floor(2.0 * u);            /* half-pitch index: even = tooth, odd = gap */
  double best = INFINITY;
  for (int m = -1; m <= 1; ++m) {
    double kk = k + (double)m;
    double u0 = 0.5 * kk, u1 = u0 + 0.5;
    /* shift the point's u into this half-pitch's period for the arc test */
    double up = u;
    int tooth = fmod(fabs(kk), 2.0) == 0.0;
    double d = arc_dist(px, pz, r, up, tooth ? r_tip : r_root, u0, u1, z, phase);
    if (d < best) best = d;
    d = flank_dist(px, pz, u0, r_root, r_tip, z, phase);
    if (d < best) best = d;
  }
  {
    double d = flank_dist(px, pz, 0.5 * (k + 2.0), r_root, r_tip, z, phase);
    if (d < best) best = d;
  }
  double fu = u - floor(u);
  int inside = r <= r_root || (r <= r_tip && fu < 0.5);
  return inside ? -best : best;
}

double ora_shape_phi(const ora_shape* s, const double* x) {
  double d[3] = {x[0] - s->center[0], x[1] - s->center[1], x[2] - s->center[2]};
  double phi;
  switch (s->kind) {
    case ORA_SHAPE_SPHERE:
      phi = sqrt(dot3(d, d)) - s->size[0];
      break;
    case ORA_SHAPE_BOX: {
      double q[3], o = 0.0, in = -INFINITY;
      for (int a = 0; a < 3; ++a) {
        q[a] = fabs(d[a]) - s->size[a];
        if (q[a] > 0.0) o += q[a] * q[a];
        if (q[a] > in) in = q[a];
      }
      phi = sqrt(o) + (in < 0.0 ? in : 0.0);
      break;
    }
    case ORA_SHAPE_CYLINDER:
      phi = extrude(len2(d[0], d[2]) - s->size[0], d[1], s->size[1]);
      break;
    case ORA_SHAPE_GEAR:
      phi = extrude(gear_section(d[0], d[2], s->teeth, s->size[0], s->size[1], s->phase), d[1], s->size[2]);
      break;
    default:
      return NAN;
  }
  return s->inside ? phi : -phi;
}

/* unit normal: central differences of phi, step eps = 1e-6 h */
void ora_shape_normal(const ora_shape* s, double eps, const double* x, double* n) {
  double g[3];
  for (int a = 0; a < 3; ++a) {
    double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
    xp[a] += eps;
    xm[a] -= eps;
    g[a] = ora_shape_phi(s, xp) - ora_shape_phi(s, xm);
  }
  double l = sqrt(dot3(g, g));
  for (int a = 0; a < 3; ++a) n[a] = l > 0.0 ? g[a] / l : 0.0;
}

/* Kernel-gradient integral over the region outside the shape, phi > 0,       */
/* seen from x: I = int_{phi(y) > 0} grad_x W(x - y) dy, by the midpoint rule */
/* on the cube [-2h, 2h]^3 around x cut into (2K)^3 cells of edge h/4, each   */
/* cell weighted by its outside volume fraction, taken linear in phi across   */
/* one cell edge: clamp(1/2 + phi/edge, 0, 1) (exact for a face-parallel     */
/* plane).                                                                    */
void ora_exterior_integral(const ora_params* P, const ora_shape* s, const double* x, double* I) {
  double h = P->h_over_dp * P->dp;
  double del = 0.25 * h;
  const int K = ORA_RELAX_QK;
  double acc[3] = {0.0, 0.0, 0.0};
  I[0] = I[1] = I[2] = 0.0;
  if (ora_shape_phi(s, x) <= -2.0 * h - del) return;   /* every cell entirely inside */
  double dv = del * del * del;
  for (int a = -K; a < K; ++a)
    for (int b = -K; b < K; ++b)
      for (int c = -K; c < K; ++c) {
        double y[3] = {x[0] + del * ((double)a + 0.5), x[1] + del * ((double)b + 0.5),
                       x[2] + del * ((double)c + 0.5)};
        double r = sqrt(dist2(x, y));
        if (r >= 2.0 * h) continue;
        /* outside volume fraction of the cell: linear in phi across one edge */
        double f = 0.5 + ora_shape_phi(s, y) / del;
        if (!(f > 0.0)) continue;
        if (f > 1.0) f = 1.0;
        double F = ora_kernel_F(r, h);        /* grad_x W(x - y) = F (x - y) */
        for (int k = 0; k < 3; ++k) acc[k] += F * (x[k] - y[k]) * (f * dv);
      }
  I[0] = acc[0];
  I[1] = acc[1];
  I[2] = acc[2];
}

/* One relaxation iteration over n particles of volume dp^3 inside the shape:
 *   F_p,i = -(2/m) sum_j V_i V_j p0 grad_i W_ij  (eq. 7), with the particles
 *           missing beyond the surface replaced by the continuum: the sum
 *           gains V_i p0 times the exterior integral (reading of the level-set
 *           compensation of the kernel deficiency);
 *   dt    = 0.25 sqrt(h / max_i |F_p,i|)         (eq. 8);
 *   x_i  += F_p,i dt^2 / 2                       (eq. 9);
 *   confinement: a particle with phi > -dp/2 after the move is put back on
 *   the level phi = -dp/2 along the normal (reading of the static level-set
 *   confinement).
 * acc (n x 3, nullable) receives F_p; stats = {max |F_p|, dt, bounded count}.
 * p0 and the density cancel in the displacement; p0 = 1 and rho0 are used.  */
int ora_relax_step(const ora_params* P, const ora_shape* s, int64_t n, double* x, double* acc,
                   double* stats) {
  double h = P->h_over_dp * P->dp;
  double V = P->dp * P->dp * P->dp, m = P->rho0 * V, p0 = 1.0;
  ora_nbr* nb = NULL;
  int rc = ora_nbr_build(P, n, x, 0, NULL, 0, &nb);
  if (rc) return rc;
  double* a = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  if (!a) { ora_nbr_free(nb); return ORA_ERR_OOM; }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    double sum[3] = {0.0, 0.0, 0.0}, I[3];
    pgeo g;
    for (int64_t p = nb->off_f[i]; p < nb->off_f[i + 1]; ++p) {
      pair_geom(nb->xb + 3 * i, nb->xb + 3 * (int64_t)nb->idx_f[p], nb->h, &g);
      for (int k = 0; k < 3; ++k) sum[k] += V * V * p0 * g.F * g.r[k];
    }
    ora_exterior_integral(P, s, x + 3 * i, I);
    for (int k = 0; k < 3; ++k) a[3 * i + k] = -(2.0 / m) * (sum[k] + V * p0 * I[k]);
  }
  double amax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double l = sqrt(dot3(a + 3 * i, a + 3 * i));
    if (l > amax) amax = l;
  }
  double dt = amax > 0.0 ? 0.25 * sqrt(h / amax) : 0.0;
  int64_t bounded = 0;
#pragma omp parallel for schedule(static) reduction(+ : bounded)
  for (int64_t i = 0; i < n; ++i) {
    double* xi = x + 3 * i;
    for (int k = 0; k < 3; ++k) xi[k] += 0.5 * a[3 * i + k] * dt * dt;
    double phi = ora_shape_phi(s, xi);
    if (phi > -0.5 * P->dp) {
      double nn[3];
      ora_shape_normal(s, 1e-6 * h, xi, nn);
      for (int k = 0; k < 3; ++k) xi[k] -= (phi + 0.5 * P->dp) * nn[k];
      bounded += 1;
    }
  }
  if (acc) memcpy(acc, a, sizeof(double) * 3 * (size_t)n);
  if (stats) { stats[0] = amax; stats[1] = dt; stats[2] = (double)bounded; }
  free(a);
  ora_nbr_free(nb);
  return ORA_OK;
}

void ora_shape_eval(const ora_shape* s, double eps, int64_t n, const double* x, double* phi, double* nrm) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    if (phi) phi[i] = ora_shape_phi(s, x + 3 * i);
    if (nrm) ora_shape_normal(s, eps, x + 3 * i, nrm + 3 * i);
  }
}

void ora_exterior_integral_n(const ora_params* P, const ora_shape* s, int64_t n, const double* x, double* I) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) ora_exterior_integral(P, s, x + 3 * i, I + 3 * i);
}
