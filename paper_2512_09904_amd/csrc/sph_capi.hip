// sph_capi.hip -- host orchestrator and C ABI of the WCSPH hot path.
//
// A pool owns up to MAX_SLOTS independent solves ("slots"), each in one
// device arena obtained from the caller's allocator.  Every advection step is
// one fixed launch sequence over the launch table of the active slots; the
// sequence is captured once per slot composition into a hipGraph and
// replayed.  A single solver is a pool with one slot.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sph_internal.h"

using namespace sphk;

static thread_local std::string g_err;
static thread_local const char* g_err_lit = nullptr;   // a message of fail_lit (no copy)

static int fail(int code, const std::string& msg) {
  g_err = msg;
  g_err_lit = nullptr;
  return code;
}

// the same for a string literal, without copying it (the allocation-free path)
static int fail_lit(int code, const char* msg) {
  g_err_lit = msg;
  return code;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(SPH_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

extern "C" const char* sph_error_string(int code) {
  switch (code) {
    case SPH_OK: return "ok";
    case SPH_ERR_ARG: return "invalid argument";
    case SPH_ERR_OOM: return "out of device memory";
    case SPH_ERR_HIP: return "HIP runtime error";
    case SPH_ERR_STATE: return "invalid state";
    case SPH_ERR_DOMAIN: return "particle left the cell grid";
    case SPH_ERR_NONFINITE: return "non-finite value in the state";
    case SPH_ERR_CAPACITY: return "neighbour row or body-accumulator capacity exceeded";
    case SPH_ERR_BUDGET: return "no free slot or HBM budget";
    default: return "unknown error";
  }
}

extern "C" const char* sph_last_error(void) { return g_err_lit ? g_err_lit : g_err.c_str(); }

// ---------------------------------------------------------------------------
// slot plan: validated sizes and the arena layout
// ---------------------------------------------------------------------------
namespace {

struct Plan {
  int prec = 0;
  int64_t nf = 0, ns = 0;
  int32_t ncells = 0, dims[3] = {0, 0, 0}, nslices = 0, kf = 0, ks = 0;
  int32_t nblk[NDOM] = {0, 0, 0, 0};
  int64_t rowlen_f = 0, rowlen_s = 0;
  int32_t nmat = 1;
  size_t pos_sz = 8, real_sz = 4, temp_sz = 8;
  size_t total = 0;
};

static size_t prec_pos(int p) { return p == SPH_PREC_FP32 ? 4 : 8; }
static size_t prec_real(int p) { return p == SPH_PREC_FP64 ? 8 : 4; }
static size_t prec_temp(int p) { return p == SPH_PREC_FP32 ? 4 : 8; }

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

static int make_plan(const sph_params* p, int prec, int64_t nf, int64_t ns, Plan* P) {
  if (!p) return fail(SPH_ERR_ARG, "params is NULL");
  if (!(p->dp > 0) || !(p->h_over_dp >= 1.0 && p->h_over_dp <= 2.0) || !(p->rho0 > 0) || !(p->c0 > 0) ||
      !(p->nu > 0) || !(p->k_f > 0) || !(p->cp_f > 0) || !(p->cfl_ad > 0) || !(p->cfl_ac > 0))
    return fail(SPH_ERR_ARG, "non-positive constant or h_over_dp outside [1, 2]");
  if (prec < 0 || prec > 2) return fail(SPH_ERR_ARG, "unknown precision");
  if (nf < 1 || nf >= (int64_t)1 << 31 || ns < 0 || ns >= (int64_t)1 << 31)
    return fail(SPH_ERR_ARG, "particle counts out of range");
  if (p->fixed_dt_ad > 0 && p->fixed_nac < 1) return fail(SPH_ERR_ARG, "fixed_nac must be >= 1");
  if (p->viscous_heating != 0 && p->viscous_heating != 1) return fail(SPH_ERR_ARG, "viscous_heating must be 0 or 1");
  if (p->wall_visc != SPH_WALL_VISC_SHEPARD && p->wall_visc != SPH_WALL_VISC_RIGID)
    return fail(SPH_ERR_ARG, "wall_visc must be SPH_WALL_VISC_SHEPARD or SPH_WALL_VISC_RIGID");
  if (p->reserved2 != 0) return fail(SPH_ERR_ARG, "reserved2 must be 0");
  if (p->n_materials < 0 || p->n_materials > SPH_MAX_MATERIALS)
    return fail(SPH_ERR_ARG, "n_materials must be in [0, 8]");
  for (int m = 0; m < p->n_materials; ++m)
    if (!(p->mat_k[m] > 0) || !(p->mat_cp[m] > 0)) return fail(SPH_ERR_ARG, "material k and cp must be > 0");
  P->nmat = p->n_materials > 1 ? p->n_materials : 1;
  const double h = p->h_over_dp * p->dp;
  const double cs = 2.0 * h;
  int64_t ncell = 1;
  for (int a = 0; a < 3; ++a) {
    const double n = std::ceil((p->grid_hi[a] - p->grid_lo[a]) / cs);
    if (!(n >= 1.0) || n > 1024.0) return fail(SPH_ERR_ARG, "grid must hold 1..1024 cells per axis");
    P->dims[a] = (int32_t)n;
    ncell *= (int64_t)n;
  }
  if (ncell > ((int64_t)1 << 26)) return fail(SPH_ERR_ARG, "grid holds more than 2^26 cells");
  P->prec = prec;
  P->nf = nf;
  P->ns = ns;
  P->ncells = (int32_t)ncell;
  // capacities are rounded up to multiples of 4 (rows are walked 4 at a time)
  // multiples of sixteen: the sweeps read whole row groups of up to 16 entries
  P->kf = ((p->max_fluid_nbrs > 0 ? p->max_fluid_nbrs : 128) + 15) & ~15;
  P->ks = ((p->max_solid_nbrs > 0 ? p->max_solid_nbrs : 96) + 15) & ~15;
  if (P->kf > 1024 || P->ks > 1024) return fail(SPH_ERR_ARG, "neighbour capacity above 1024");
  P->nslices = (int32_t)ceil_div(nf, WAVE);
  P->rowlen_f = (int64_t)P->nslices * P->kf * WAVE;
  P->rowlen_s = (int64_t)P->nslices * P->ks * WAVE;
  P->nblk[DOM_FLUID] = (int32_t)ceil_div(nf, BLOCK);
  P->nblk[DOM_SOLID] = (int32_t)ceil_div(ns, BLOCK);
  P->nblk[DOM_CELL] = (int32_t)ceil_div(ncell, BLOCK);
  P->nblk[DOM_SLOT] = 1;
  P->pos_sz = prec_pos(prec);
  P->real_sz = prec_real(prec);
  P->temp_sz = prec_temp(prec);
  return SPH_OK;
}

// Walks the arena layout; with base == nullptr it only sums the sizes.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <class T>
  void take(T*& ptr, size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    ptr = base ? (T*)(base + off) : nullptr;
    off += bytes;
  }
  void takev(void*& ptr, size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    ptr = base ? (void*)(base + off) : nullptr;
    off += bytes;
  }
};

static size_t carve(const Plan& P, void* base, SlotDesc* d) {
  SlotDesc tmp;
  SlotDesc& D = d ? *d : tmp;
  Carver C(base);
  const size_t nf = (size_t)P.nf, ns = (size_t)P.ns, nc = (size_t)P.ncells;
  const size_t ps = P.pos_sz, rs = P.real_sz, ts = P.temp_sz;
  const size_t nbf = (size_t)P.nblk[DOM_FLUID], nbc = (size_t)P.nblk[DOM_CELL];
  C.take(D.ctl, sizeof(SlotCtl));
  C.takev(D.xa, 4 * nf * ps);
  C.takev(D.drift, 4 * nf * rs);
  C.takev(D.vr, 4 * nf * rs);
  C.takev(D.vrn, 4 * nf * rs);
  C.takev(D.drho, nf * rs);
  C.takev(D.T, nf * ts);
  C.takev(D.td, 16 * nf);
  C.takev(D.ah, 4 * nf * rs);
  C.take(D.fid, nf * 4);
  C.take(D.sumW, nf * 8);
  C.take(D.fcell, nf * 4);
  C.take(D.fperm, nf * 4);
  C.take(D.fkey, nf * 8);
  C.takev(D.xa2, 4 * nf * ps);
  C.takev(D.vr2, 4 * nf * rs);
  C.takev(D.drho2, nf * rs);
  C.takev(D.T2, nf * ts);
  C.take(D.fid2, nf * 4);
  if (P.nmat > 1) {
    C.take(D.mat, nf * 4);
    C.take(D.mat2, nf * 4);
  }
  C.take(D.nfc, nf * 4);
  C.take(D.nsc, nf * 4);
  C.take(D.nrec, 4 * (size_t)P.rowlen_f);
  C.take(D.srec, 4 * (size_t)P.rowlen_s);
  C.take(D.rmaj, 4 * nf * (size_t)(P.kf + P.ks));
  C.takev(D.xo, 4 * nf * rs);
  C.takev(D.so, 4 * ns * rs);
  C.takev(D.x0, ns * 32);
  C.takev(D.n0, ns * 32);
  C.take(D.body, ns * 4);
  C.take(D.sid, ns * 4);
  C.takev(D.xw, 4 * ns * ps);
  C.takev(D.nw, 4 * ns * rs);
  C.takev(D.vw, 4 * ns * rs);
  C.takev(D.lev, 4 * ns * rs);
  C.takev(D.x0b, ns * 32);
  C.takev(D.n0b, ns * 32);
  C.take(D.bodyb, ns * 4);
  C.take(D.sidb, ns * 4);
  C.takev(D.xwb, 4 * ns * ps);
  C.takev(D.nwb, 4 * ns * rs);
  C.takev(D.vwb, 4 * ns * rs);
  C.takev(D.levb, 4 * ns * rs);
  C.take(D.scell, ns * 4);
  C.take(D.sperm, ns * 4);
  C.take(D.zeta, ns * 8);
  C.takev(D.vd, 4 * ns * rs);
  C.take(D.skey, ns * 8);
  C.take(D.rank, nc * 4);
  C.take(D.cnt_f, nc * 4);
  C.take(D.cnt_s, nc * 4);
  C.take(D.start_f, (nc + 1) * 4);
  C.take(D.start_s, (nc + 1) * 4);
  C.take(D.bsum_f, nbc * 4);
  C.take(D.bsum_s, nbc * 4);
  C.take(D.vmax_part, nbf * 8);
  C.take(D.visc_part, nbf * NB * 7 * 8);
  C.take(D.press_part, nbf * NB * 6 * 8);
  C.take(D.glob_part, nbf * (NGLOB + 1) * 8);
  return (C.off + 255) & ~(size_t)255;
}

static uint32_t morton3(uint32_t cx, uint32_t cy, uint32_t cz) {
  uint32_t k = 0;
  for (int b = 0; b < 10; ++b) {
    k |= ((cx >> b) & 1u) << (3 * b);
    k |= ((cy >> b) & 1u) << (3 * b + 1);
    k |= ((cz >> b) & 1u) << (3 * b + 2);
  }
  return k;
}

// rank of each cell (row-major linear index) in Morton order, and its inverse
static void rank_table(const int32_t dims[3], std::vector<uint32_t>& rank, std::vector<uint32_t>& morton_of_rank) {
  const int64_t n = (int64_t)dims[0] * dims[1] * dims[2];
  std::vector<uint64_t> key((size_t)n);
  for (int32_t z = 0; z < dims[2]; ++z)
    for (int32_t y = 0; y < dims[1]; ++y)
      for (int32_t x = 0; x < dims[0]; ++x) {
        const int64_t lin = ((int64_t)z * dims[1] + y) * dims[0] + x;
        key[(size_t)lin] = ((uint64_t)morton3((uint32_t)x, (uint32_t)y, (uint32_t)z) << 32) | (uint64_t)lin;
      }
  std::sort(key.begin(), key.end());
  rank.assign((size_t)n, 0u);
  morton_of_rank.assign((size_t)n, 0u);
  for (int64_t r = 0; r < n; ++r) {
    rank[(size_t)(key[(size_t)r] & 0xffffffffu)] = (uint32_t)r;
    morton_of_rank[(size_t)r] = (uint32_t)(key[(size_t)r] >> 32);
  }
}

// perfect-lattice kernel sum dp^3 sum W (self included), the reference of eq. 14
static double lattice_sum0(double hod) {
  const double a = 21.0 / (16.0 * M_PI * hod * hod * hod);
  const int R = (int)std::ceil(2.0 * hod) + 1;
  double s = 0.0;
  for (int i = -R; i <= R; ++i)
    for (int j = -R; j <= R; ++j)
      for (int k = -R; k <= R; ++k) {
        const double q = std::sqrt((double)(i * i + j * j + k * k)) / hod;
        if (q >= 2.0) continue;
        const double t = 1.0 - 0.5 * q;
        s += a * t * t * t * t * (1.0 + 2.0 * q);
      }
  return s;
}

// Perfect-lattice kernel sum (units of dp^3) over the sites with x > 0 seen
// from a site on x = 0: the full-immersion reference of the contact factor.
static double lattice_halfspace(double hod) {
  const double a = 21.0 / (16.0 * M_PI * hod * hod * hod);
  const int R = (int)std::ceil(2.0 * hod) + 1;
  double s = 0.0;
  for (int i = 1; i <= R; ++i)
    for (int j = -R; j <= R; ++j)
      for (int k = -R; k <= R; ++k) {
        const double q = std::sqrt((double)(i * i + j * j + k * k)) / hod;
        if (q >= 2.0) continue;
        const double t = 1.0 - 0.5 * q;
        s += a * t * t * t * t * (1.0 + 2.0 * q);
      }
  return s;
}

// Sub-steps per advection step can never exceed this for |v|max in
// [tip speed, c0] (eq. 25); launches beyond a slot's n_ac exit at once.
static int nac_bound(const sph_params* p, double vtip) {
  if (p->fixed_dt_ad > 0) return std::max(1, p->fixed_nac);
  const double h = p->h_over_dp * p->dp;
  auto n_of = [&](double vm) {
    const double visc = h * h / p->nu;
    const double adv = vm > 0.0 ? h / vm : visc;
    const double tad = p->cfl_ad * (adv < visc ? adv : visc);
    const double tac = p->cfl_ac * h / (p->c0 + vm);
    return std::ceil(tad / tac * (1.0 + 1e-9));
  };
  double n = n_of(vtip);
  const double vstar = p->nu / h;
  if (vstar > vtip && vstar < p->c0) n = std::max(n, n_of(vstar));
  n = std::max(n, n_of(p->c0));
  const int cap = p->nac_max > 0 ? p->nac_max : 16;
  return (int)std::max(1.0, std::min(n, (double)cap));
}

struct SlotHost {
  bool used = false;
  Plan plan;
  SlotDesc d;
  void* arena = nullptr;
  size_t bytes = 0;
  sph_params params;
  int32_t nbody = 0;
  sph_body bodies[NB];
  int64_t target = 0, launched = 0;
  bool held = false;               // left out of pool steps until resumed
  hipEvent_t ev_done = nullptr;
  bool ev_recorded = false;
  hipEvent_t ev_admit = nullptr;   // the slot's upload has completed on the main stream
  std::vector<uint32_t> morton_of_rank;
  // host sources of the slot's stream-ordered uploads: they must outlive the
  // copies, so neither is resized or reassigned while the slot is admitted
  std::vector<char> staging;
  SlotCtl ctl_staged{};
};

struct TimedLaunch {
  int kid;
  hipEvent_t a, b;
};

}  // namespace

struct sph_pool {
  hipStream_t stream = nullptr;
  hipStream_t copy_stream = nullptr;
  // a second compute stream, forked from and joined back into `stream`, so
  // that the solid-centric dummy-velocity sweep overlaps the kernel sums
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  sph_allocator alloc{};
  int prec = 0;
  size_t budget = 0, used = 0;
  int max_slots = 1;
  SlotDesc* d_table = nullptr;
  SlotHost slots[MAX_SLOTS];
  bool use_graph = true, timing = false, comp_dirty = true;
  bool fuse_first = true;   // sub-step 0's half update and momentum inside the viscous/heat sweep
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  LaunchTab tab{};
  int nac_launch = 1;
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> free_events;
  std::vector<float> times[SPH_K_COUNT];
};

struct sph_solver {
  sph_pool* pool = nullptr;
  sph_params p{};
  bool inited = false;
  int32_t nbody = 0;
  sph_body bodies[NB];
  std::vector<double> x, v, rho, T, x0, n0;
  std::vector<int32_t> material;
  std::vector<int32_t> body;
  int64_t nf = 0, ns = 0;
};

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
// Every device allocation goes through the caller's allocator (the pool
// refuses to be created without one); the library never allocates by itself.
static void* dev_alloc(sph_pool* P, size_t bytes) {
  if (bytes == 0) bytes = 256;
  return P->alloc.alloc(bytes, (void*)P->stream, P->alloc.user);
}

static void dev_free(sph_pool* P, void* ptr) {
  if (!ptr) return;
  P->alloc.free(ptr, (void*)P->stream, P->alloc.user);
}

static void drop_graph(sph_pool* P) {
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->gexec = nullptr;
  P->graph = nullptr;
}

// ---------------------------------------------------------------------------
// launch sequence
// ---------------------------------------------------------------------------
static int launch(sph_pool* P, const LaunchTab& tab, int kid, int which, int sub, hipStream_t st) {
  hipEvent_t a = nullptr, b = nullptr;
  if (P->timing) {
    for (hipEvent_t* e : {&a, &b}) {
      if (!P->free_events.empty()) {
        *e = P->free_events.back();
        P->free_events.pop_back();
      } else {
        HIPCHK(hipEventCreate(e));
      }
    }
    HIPCHK(hipEventRecord(a, st));
  }
  hipError_t e = launch_kernel(P->prec, kid, which, sub, P->d_table, tab, st);
  if (e != hipSuccess) return fail(SPH_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  if (P->timing) {
    HIPCHK(hipEventRecord(b, st));
    P->pending.push_back({kid, a, b});
  }
  return SPH_OK;
}

static int launch(sph_pool* P, const LaunchTab& tab, int kid, int which, int sub) {
  return launch(P, tab, kid, which, sub, P->stream);
}

static int launch_rx(sph_pool* P, const LaunchTab& tab, int kid, int iter, const RelaxShape& g) {
  hipEvent_t a = nullptr, b = nullptr;
  if (P->timing) {
    for (hipEvent_t* e : {&a, &b}) {
      if (!P->free_events.empty()) {
        *e = P->free_events.back();
        P->free_events.pop_back();
      } else {
        HIPCHK(hipEventCreate(e));
      }
    }
    HIPCHK(hipEventRecord(a, P->stream));
  }
  hipError_t e = launch_relax(P->prec, kid, iter, P->d_table, tab, g, P->stream);
  if (e != hipSuccess) return fail(SPH_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  if (P->timing) {
    HIPCHK(hipEventRecord(b, P->stream));
    P->pending.push_back({kid, a, b});
  }
  return SPH_OK;
}

#define LCHK(x)            \
  do {                     \
    int r_ = (x);          \
    if (r_) return r_;     \
  } while (0)

// the main stream waits for the side stream's dummy velocities
static int join_side(sph_pool* P) {
  if (hipStreamWaitEvent(P->stream, P->ev_join, 0) != hipSuccess)
    return fail_lit(SPH_ERR_HIP, "join from the side stream failed");
  return SPH_OK;
}

// timed = false: no event timing and no heap allocation on success (the
// allocation-free entry point); wallvel = false: no dummy velocities (calls
// between steps that do not step: the next step's own build recomputes them);
// join = false: the caller joins the side stream itself (join_side) before
// the first kernel that reads the dummy velocities
static int enqueue_sort_build(sph_pool* P, const LaunchTab& T, bool timed = true, bool wallvel = true,
                              bool join = true) {
  auto LS = [&](int kid, int which, hipStream_t st) {
    if (timed) return launch(P, T, kid, which, 0, st);
    if (launch_kernel(P->prec, kid, which, 0, P->d_table, T, st) != hipSuccess)
      return fail_lit(SPH_ERR_HIP, "kernel launch failed");
    return (int)SPH_OK;
  };
  auto L = [&](int kid, int which) { return LS(kid, which, P->stream); };
  LCHK(L(SPH_K_CLEAR, 0));
  LCHK(L(SPH_K_POSE, 1));
  LCHK(L(SPH_K_FOLD, 0));
  LCHK(L(SPH_K_SCAN1, 0));
  LCHK(L(SPH_K_SCAN2, 0));
  LCHK(L(SPH_K_SCAN3, 0));
  LCHK(L(SPH_K_SCATTER, 0));
  LCHK(L(SPH_K_SCATTER, 1));
  LCHK(L(SPH_K_CELLSORT, 0));
  LCHK(L(SPH_K_CELLSORT, 1));
  LCHK(L(SPH_K_REORDER, 0));
  LCHK(L(SPH_K_REORDER, 1));
  LCHK(L(SPH_K_BUILD, 0));
  if (!wallvel) {
    LCHK(L(SPH_K_SUMW, 0));
    return SPH_OK;
  }
  // the dummy velocities (solids) on the side stream, beside the kernel sums
  // (fluid): both read the fresh build, neither reads the other's output
  if (hipEventRecord(P->ev_fork, P->stream) != hipSuccess ||
      hipStreamWaitEvent(P->side_stream, P->ev_fork, 0) != hipSuccess)
    return fail_lit(SPH_ERR_HIP, "fork to the side stream failed");
  LCHK(LS(SPH_K_WALLVEL, 1, P->side_stream));
  if (hipEventRecord(P->ev_join, P->side_stream) != hipSuccess)
    return fail_lit(SPH_ERR_HIP, "event record on the side stream failed");
  LCHK(L(SPH_K_SUMW, 0));
  return join ? join_side(P) : (int)SPH_OK;
}

static int enqueue_step(sph_pool* P, const LaunchTab& T, int nac) {
  LCHK(enqueue_sort_build(P, T, true, true, false));
  LCHK(launch(P, T, SPH_K_DT, 0, 0));   // reads no dummy velocity: runs beside them
  LCHK(join_side(P));
  // sub-step s: momentum, then continuity, which also closes s and opens
  // s + 1; the viscous/heat sweep runs sub-step 0's opening half and momentum
  // (unfused: their own launches, the same arithmetic)
  int s0 = 0;
  if (P->fuse_first) {
    LCHK(launch(P, T, SPH_K_VISC_HEAT, 1, 0));
    LCHK(launch(P, T, SPH_K_CONTINUITY, 0, 0));
    s0 = 1;
  } else {
    LCHK(launch(P, T, SPH_K_VISC_HEAT, 0, 0));
    LCHK(launch(P, T, SPH_K_HALF_A, 0, 0));
  }
  for (int s = s0; s < nac; ++s) {
    LCHK(launch(P, T, SPH_K_MOMENTUM, 0, s));
    LCHK(launch(P, T, SPH_K_CONTINUITY, 0, s));
  }
  LCHK(launch(P, T, SPH_K_END, 0, 0));
  LCHK(launch(P, T, SPH_K_FINAL, 0, 0));
  return SPH_OK;
}

// the launch table of slot `slot` alone (no heap allocation)
static void tab_one(sph_pool* P, int slot, LaunchTab& T) {
  std::memset(&T, 0, sizeof(T));
  T.n = 1;
  T.slot[0] = slot;
  if (P->slots[slot].d.diss) T.flags |= TAB_DISS;
  if (P->slots[slot].d.nmat > 1) T.flags |= TAB_MAT;
  for (int d = 0; d < NDOM; ++d) T.blk0[d][1] = P->slots[slot].plan.nblk[d];
}

static void tab_for(sph_pool* P, const std::vector<int>& slots, LaunchTab& T) {
  std::memset(&T, 0, sizeof(T));
  T.n = (int32_t)slots.size();
  for (int d = 0; d < NDOM; ++d) T.blk0[d][0] = 0;
  for (size_t k = 0; k < slots.size(); ++k) {
    T.slot[k] = slots[k];
    if (P->slots[slots[k]].d.diss) T.flags |= TAB_DISS;
    if (P->slots[slots[k]].d.nmat > 1) T.flags |= TAB_MAT;
    const Plan& pl = P->slots[slots[k]].plan;
    for (int d = 0; d < NDOM; ++d) T.blk0[d][k + 1] = T.blk0[d][k] + pl.nblk[d];
  }
}

static void recompose(sph_pool* P) {
  std::vector<int> act;
  int nac = 1;
  for (int s = 0; s < P->max_slots; ++s) {
    const SlotHost& S = P->slots[s];
    if (S.used && !S.held && S.launched < S.target) {
      act.push_back(s);
      nac = std::max(nac, S.d.nac_bound);
    }
  }
  tab_for(P, act, P->tab);
  P->nac_launch = nac;
  drop_graph(P);
  P->comp_dirty = false;
}

static int collect_timing(sph_pool* P) {
  if (P->pending.empty()) return SPH_OK;
  HIPCHK(hipStreamSynchronize(P->stream));
  for (const TimedLaunch& t : P->pending) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t.a, t.b));
    P->times[t.kid].push_back(ms);
    P->free_events.push_back(t.a);
    P->free_events.push_back(t.b);
  }
  P->pending.clear();
  return SPH_OK;
}

// ---------------------------------------------------------------------------
// pool
// ---------------------------------------------------------------------------
extern "C" size_t sph_bytes_required(const sph_params* p, int64_t nf, int64_t ns) {
  Plan P;
  if (make_plan(p, p ? p->precision : 0, nf, ns, &P)) return 0;
  return carve(P, nullptr, nullptr);
}

extern "C" int sph_pool_create(size_t budget, int32_t max_slots, int32_t precision,
                               const sph_allocator* a, void* stream, sph_pool** out) {
  if (!out) return fail(SPH_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > MAX_SLOTS) return fail(SPH_ERR_ARG, "max_slots must be in [1, 32]");
  if (precision < 0 || precision > 2) return fail(SPH_ERR_ARG, "unknown precision");
  if (!a || !a->alloc || !a->free) return fail(SPH_ERR_ARG, "an allocator with alloc and free is required");
  sph_pool* P = new sph_pool();
  P->stream = (hipStream_t)stream;
  P->alloc = *a;
  P->prec = precision;
  P->budget = budget;
  P->max_slots = max_slots;
  P->use_graph = stream != nullptr;
  // default stream priority for both (streams of different priorities are avoided)
  if (hipStreamCreateWithFlags(&P->copy_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&P->side_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming) != hipSuccess) {
    if (P->copy_stream) (void)hipStreamDestroy(P->copy_stream);
    if (P->side_stream) (void)hipStreamDestroy(P->side_stream);
    if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
    if (P->ev_join) (void)hipEventDestroy(P->ev_join);
    delete P;
    return fail(SPH_ERR_HIP, "stream or event creation failed");
  }
  P->d_table = (SlotDesc*)dev_alloc(P, sizeof(SlotDesc) * MAX_SLOTS);
  if (!P->d_table) {
    (void)hipStreamDestroy(P->copy_stream);
    (void)hipStreamDestroy(P->side_stream);
    (void)hipEventDestroy(P->ev_fork);
    (void)hipEventDestroy(P->ev_join);
    delete P;
    return fail(SPH_ERR_OOM, "slot table allocation failed");
  }
  *out = P;
  return SPH_OK;
}

template <class T>
static void put(std::vector<char>& buf, size_t off, T val) {
  std::memcpy(buf.data() + off, &val, sizeof(T));
}

// host copies converted to the device layout of a slot
static int upload_slot(sph_pool* P, SlotHost& S, const double* x, const double* v, const double* rho,
                       const double* T, const int32_t* material, const double* x0, const double* n0,
                       const int32_t* body) {
  const Plan& pl = S.plan;
  const size_t nf = (size_t)pl.nf, ns = (size_t)pl.ns;
  const size_t ps = pl.pos_sz, rs = pl.real_sz, ts = pl.temp_sz;
  const double rho0 = S.params.rho0;
  const bool rel = pl.prec != SPH_PREC_FP32;
  std::vector<uint32_t> rank;
  rank_table(pl.dims, rank, S.morton_of_rank);
  // staging: xa (x,y,z,0) | vr (vx,vy,vz,rho) | T | fid | x0 (x,y,z,0) | n0 | body | sid | rank
  const size_t nm = pl.nmat > 1 ? nf : 0;
  const size_t o_xa = 0, o_v = o_xa + 4 * nf * ps, o_T = o_v + 4 * nf * rs, o_fid = o_T + nf * ts,
               o_mat = o_fid + nf * 4, o_x0 = o_mat + nm * 4, o_n0 = o_x0 + ns * 32, o_b = o_n0 + ns * 32,
               o_sid = o_b + ns * 4, o_rank = o_sid + ns * 4, o_end = o_rank + rank.size() * 4;
  S.staging.assign(o_end, 0);
  std::vector<char>& B = S.staging;
  auto put_real = [&](size_t off, size_t sz, size_t idx, double val) {
    if (sz == 8) put<double>(B, off + idx * 8, val);
    else put<float>(B, off + idx * 4, (float)val);
  };
  for (size_t i = 0; i < nf; ++i) {
    for (size_t k = 0; k < 3; ++k) {
      put_real(o_xa, ps, 4 * i + k, x[3 * i + k]);
      put_real(o_v, rs, 4 * i + k, v ? v[3 * i + k] : 0.0);
    }
    put_real(o_v, rs, 4 * i + 3, rel ? rho[i] - rho0 : rho[i]);
    put_real(o_T, ts, i, T[i]);
    put<uint32_t>(B, o_fid + i * 4, (uint32_t)i);
    if (nm) put<uint32_t>(B, o_mat + i * 4, material ? (uint32_t)material[i] : 0u);
  }
  for (size_t w = 0; w < ns; ++w) {
    for (size_t k = 0; k < 3; ++k) {
      put<double>(B, o_x0 + (4 * w + k) * 8, x0[3 * w + k]);
      put<double>(B, o_n0 + (4 * w + k) * 8, n0[3 * w + k]);
    }
    put<int32_t>(B, o_b + w * 4, body[w]);
    put<uint32_t>(B, o_sid + w * 4, (uint32_t)w);
  }
  std::memcpy(B.data() + o_rank, rank.data(), rank.size() * 4);
  hipStream_t st = P->stream;
  const SlotDesc& D = S.d;
  HIPCHK(hipMemsetAsync(S.arena, 0, S.bytes, st));
  HIPCHK(hipMemcpyAsync(D.xa, B.data() + o_xa, 4 * nf * ps, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(D.vr, B.data() + o_v, 4 * nf * rs, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(D.T, B.data() + o_T, nf * ts, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(D.fid, B.data() + o_fid, nf * 4, hipMemcpyHostToDevice, st));
  if (nm) HIPCHK(hipMemcpyAsync(D.mat, B.data() + o_mat, nf * 4, hipMemcpyHostToDevice, st));
  if (ns) {
    HIPCHK(hipMemcpyAsync(D.x0, B.data() + o_x0, ns * 32, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(D.n0, B.data() + o_n0, ns * 32, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(D.body, B.data() + o_b, ns * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(D.sid, B.data() + o_sid, ns * 4, hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(D.rank, B.data() + o_rank, rank.size() * 4, hipMemcpyHostToDevice, st));
  return SPH_OK;
}

static int admit(sph_pool* P, const sph_params* p, int32_t nbody, const sph_body* b, int64_t nf,
                 const double* x, const double* v, const double* rho, const double* T, const int32_t* material,
                 int64_t ns, const double* x0, const double* n0, const int32_t* body, int64_t target,
                 int32_t* slot_out) {
  if (!P || !slot_out) return fail(SPH_ERR_ARG, "NULL pool or slot");
  if (nbody < 1 || nbody > NB || !b) return fail(SPH_ERR_ARG, "need 1..8 bodies");
  if (!x || !rho || !T) return fail(SPH_ERR_ARG, "fluid arrays missing");
  if (ns > 0 && (!x0 || !n0 || !body)) return fail(SPH_ERR_ARG, "solid arrays missing");
  if (target < 1) return fail(SPH_ERR_ARG, "target_steps must be >= 1");
  Plan pl;
  int rc = make_plan(p, P->prec, nf, ns, &pl);
  if (rc) return rc;
  for (int64_t w = 0; w < ns; ++w)
    if (body[w] < 0 || body[w] >= nbody) return fail(SPH_ERR_ARG, "solid body index out of range");
  if (material)
    for (int64_t i = 0; i < nf; ++i)
      if (material[i] < 0 || material[i] >= pl.nmat) return fail(SPH_ERR_ARG, "material index out of range");
  for (int k = 0; k < nbody; ++k) {
    const double an = std::sqrt(b[k].axis[0] * b[k].axis[0] + b[k].axis[1] * b[k].axis[1] + b[k].axis[2] * b[k].axis[2]);
    if (!(an > 0) || !(b[k].k > 0)) return fail(SPH_ERR_ARG, "body axis must be non-zero and k > 0");
  }
  const size_t bytes = carve(pl, nullptr, nullptr);
  int s = -1;
  for (int k = 0; k < P->max_slots; ++k)
    if (!P->slots[k].used) {
      s = k;
      break;
    }
  if (s < 0 || P->used + bytes > P->budget) return fail(SPH_ERR_BUDGET, "no free slot or budget");
  SlotHost& S = P->slots[s];
  S = SlotHost();
  S.plan = pl;
  S.params = *p;
  S.bytes = bytes;
  S.arena = dev_alloc(P, bytes);
  if (!S.arena) return fail(SPH_ERR_OOM, "slot arena allocation failed");
  std::memset(&S.d, 0, sizeof(SlotDesc));
  carve(pl, S.arena, &S.d);
  SlotDesc& D = S.d;
  D.nf = (int32_t)nf;
  D.ns = (int32_t)ns;
  D.ncells = pl.ncells;
  D.nslices = pl.nslices;
  D.kf = pl.kf;
  D.ks = pl.ks;
  D.nbody = nbody;
  for (int a = 0; a < 3; ++a) D.dims[a] = pl.dims[a];
  D.free_surface = p->free_surface ? 1 : 0;
  D.diss = p->viscous_heating;
  D.wall_rigid = p->wall_visc == SPH_WALL_VISC_RIGID ? 1 : 0;
  D.fixed_nac = p->fixed_nac;
  for (int d = 0; d < NDOM; ++d) D.nblk[d] = pl.nblk[d];
  D.rowlen_f = pl.rowlen_f;
  D.rowlen_s = pl.rowlen_s;
  D.dp = p->dp;
  D.h = p->h_over_dp * p->dp;
  D.rho0 = p->rho0;
  D.c0 = p->c0;
  D.nu = p->nu;
  D.eta = p->rho0 * p->nu;
  // one material: k_f, cp_f (or the table's only entry); several: the table
  D.k_f = p->n_materials >= 1 ? p->mat_k[0] : p->k_f;
  D.cp_f = p->n_materials >= 1 ? p->mat_cp[0] : p->cp_f;
  D.nmat = pl.nmat;
  D.dt_T = INFINITY;
  for (int m = 0; m < NMAT; ++m) {
    D.mk[m] = m < pl.nmat && p->n_materials > 0 ? p->mat_k[m] : D.k_f;
    D.mcp[m] = m < pl.nmat && p->n_materials > 0 ? p->mat_cp[m] : D.cp_f;
    // eq. 26 with rho read as rho0
    const double hh = p->h_over_dp * p->dp;
    if (m < pl.nmat) D.dt_T = std::min(D.dt_T, 0.5 * p->rho0 * D.mcp[m] * hh * hh / D.mk[m]);
  }
  D.mass = p->rho0 * (p->dp * p->dp * p->dp);
  D.vol_w = p->dp * p->dp * p->dp;
  D.S0 = lattice_sum0(p->h_over_dp);
  D.zref = lattice_halfspace(p->h_over_dp);
  {
    const double two_h = 2.0 * D.h;
    D.cut2 = two_h * two_h;
    D.cs = 2.0 * D.h;
    D.cs_r = pl.real_sz == 8 ? D.cs : (double)(float)D.cs;
  }
  D.cfl_ad = p->cfl_ad;
  D.cfl_ac = p->cfl_ac;
  D.fixed_dt_ad = p->fixed_dt_ad;
  for (int a = 0; a < 3; ++a) {
    D.g[a] = p->gravity[a];
    D.lo[a] = p->grid_lo[a];
  }
  D.kW = 21.0 / (16.0 * M_PI * D.h * D.h * D.h);
  D.kF = -5.0 * D.kW / (D.h * D.h);
  double vtip = 0.0;
  std::vector<double> rmax((size_t)nbody, 0.0);
  for (int k = 0; k < nbody; ++k) {
    S.bodies[k] = b[k];
    const double an = std::sqrt(b[k].axis[0] * b[k].axis[0] + b[k].axis[1] * b[k].axis[1] + b[k].axis[2] * b[k].axis[2]);
    for (int a = 0; a < 3; ++a) {
      D.bc[k][a] = b[k].center[a];
      D.ba[k][a] = b[k].axis[a] / an;
    }
    D.bom[k] = b[k].omega;
    D.bT[k] = b[k].T;
    D.bk[k] = b[k].k;
  }
  S.nbody = nbody;
  for (int64_t w = 0; w < ns; ++w) {
    const int k = body[w];
    double u[3], au = 0.0;
    for (int a = 0; a < 3; ++a) {
      u[a] = x0[3 * w + a] - D.bc[k][a];
      au += D.ba[k][a] * u[a];
    }
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double d = u[a] - au * D.ba[k][a];
      d2 += d * d;
    }
    rmax[(size_t)k] = std::max(rmax[(size_t)k], std::sqrt(d2));
  }
  for (int k = 0; k < nbody; ++k) {
    D.btip[k] = b[k].omega != 0.0 ? std::fabs(b[k].omega) * rmax[(size_t)k] : 0.0;
    vtip = std::max(vtip, D.btip[k]);
  }
  D.nac_bound = nac_bound(p, vtip);
  S.target = target;
  S.launched = 0;
  rc = upload_slot(P, S, x, v, rho, T, material, x0, n0, body);
  if (rc) {
    dev_free(P, S.arena);
    S = SlotHost();
    return rc;
  }
  // the control block and table entry are copied from host memory that lives
  // as long as the slot (the copies are stream-ordered)
  std::memset(&S.ctl_staged, 0, sizeof(SlotCtl));
  S.ctl_staged.target = target;
  HIPCHK(hipMemcpyAsync(D.ctl, &S.ctl_staged, sizeof(SlotCtl), hipMemcpyHostToDevice, P->stream));
  HIPCHK(hipMemcpyAsync(P->d_table + s, &S.d, sizeof(SlotDesc), hipMemcpyHostToDevice, P->stream));
  HIPCHK(hipEventCreateWithFlags(&S.ev_done, hipEventDisableTiming));
  // polls read the control block on the copy stream; they must not see the
  // arena's earlier contents before the zeroed block has landed
  HIPCHK(hipEventCreateWithFlags(&S.ev_admit, hipEventDisableTiming));
  HIPCHK(hipEventRecord(S.ev_admit, P->stream));
  S.used = true;
  P->used += bytes;
  P->comp_dirty = true;
  *slot_out = s;
  return SPH_OK;
}

extern "C" int sph_pool_admit(sph_pool* P, const sph_params* p, int32_t nbody, const sph_body* b, int64_t nf,
                              const double* x, const double* v, const double* rho, const double* T,
                              const int32_t* material, int64_t ns, const double* x0, const double* n0,
                              const int32_t* body, int64_t target_steps, int32_t* slot) {
  return admit(P, p, nbody, b, nf, x, v, rho, T, material, ns, x0, n0, body, target_steps, slot);
}

static int pool_step(sph_pool* P, int32_t n) {
  if (!P) return fail(SPH_ERR_ARG, "NULL pool");
  if (n < 0) return fail(SPH_ERR_ARG, "negative step count");
  if (P->comp_dirty) recompose(P);
  if (P->tab.n == 0 || n == 0) return SPH_OK;
  const bool graph = P->use_graph && !P->timing;
  for (int k = 0; k < n; ++k) {
    if (graph) {
      if (!P->gexec) {
        HIPCHK(hipStreamBeginCapture(P->stream, hipStreamCaptureModeRelaxed));
        int rc = enqueue_step(P, P->tab, P->nac_launch);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(P->stream, &g);
        if (rc) {
          if (g) (void)hipGraphDestroy(g);
          return rc;
        }
        if (e != hipSuccess) return fail(SPH_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        P->graph = g;
        HIPCHK(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
      }
      HIPCHK(hipGraphLaunch(P->gexec, P->stream));
    } else {
      LCHK(enqueue_step(P, P->tab, P->nac_launch));
    }
  }
  bool finished = false;
  for (int k = 0; k < P->tab.n; ++k) {
    SlotHost& S = P->slots[P->tab.slot[k]];
    S.launched += n;
    if (S.launched >= S.target && !S.ev_recorded) {
      HIPCHK(hipEventRecord(S.ev_done, P->stream));
      S.ev_recorded = true;
      finished = true;
    }
  }
  if (finished) P->comp_dirty = true;
  return SPH_OK;
}

extern "C" int sph_pool_step(sph_pool* P, int32_t n) { return pool_step(P, n); }

extern "C" int sph_pool_hold(sph_pool* P, int32_t slot, int32_t hold) {
  if (!P || slot < 0 || slot >= P->max_slots || !P->slots[slot].used) return fail(SPH_ERR_ARG, "bad slot");
  if (hold != 0 && hold != 1) return fail(SPH_ERR_ARG, "hold must be 0 or 1");
  SlotHost& S = P->slots[slot];
  if (S.held != (hold == 1)) {
    S.held = hold == 1;
    P->comp_dirty = true;
  }
  return SPH_OK;
}

static int read_ctl(sph_pool* P, SlotHost& S, SlotCtl* ctl, bool sync_main) {
  if (sync_main) {
    HIPCHK(hipStreamSynchronize(P->stream));
    HIPCHK(hipMemcpy(ctl, S.d.ctl, sizeof(SlotCtl), hipMemcpyDeviceToHost));
  } else {
    HIPCHK(hipMemcpyAsync(ctl, S.d.ctl, sizeof(SlotCtl), hipMemcpyDeviceToHost, P->copy_stream));
    HIPCHK(hipStreamSynchronize(P->copy_stream));
  }
  return SPH_OK;
}

static int flag_code(uint32_t f) {
  if (f & F_NONFINITE) return SPH_ERR_NONFINITE;
  if (f & F_DOMAIN) return SPH_ERR_DOMAIN;
  if (f & F_CAPACITY) return SPH_ERR_CAPACITY;
  return SPH_OK;
}

static void fill_reports(const SlotHost& S, const SlotCtl& c, sph_report* r, sph_body_report* br) {
  if (r) {
    *r = c.rep;
    r->flags = (int32_t)c.flags;
    r->t = c.t;
    r->step = c.step;
  }
  if (br)
    for (int b = 0; b < S.nbody; ++b) br[b] = c.brep[b];
}

extern "C" int sph_pool_poll(sph_pool* P, int32_t slot, int32_t* done, sph_report* r, sph_body_report* br) {
  if (!P || slot < 0 || slot >= P->max_slots || !P->slots[slot].used || !done)
    return fail(SPH_ERR_ARG, "bad slot");
  SlotHost& S = P->slots[slot];
  *done = 0;
  SlotCtl c;
  bool complete = false;
  if (S.ev_recorded) {
    hipError_t q = hipEventQuery(S.ev_done);
    if (q == hipSuccess) complete = true;
    else if (q != hipErrorNotReady) return fail(SPH_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
  }
  // until the slot's upload has run, its control block holds whatever the
  // reused memory held before: nothing to read yet
  {
    const hipError_t q = hipEventQuery(S.ev_admit);
    if (q == hipErrorNotReady) return SPH_OK;
    if (q != hipSuccess) return fail(SPH_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
  }
  LCHK(read_ctl(P, S, &c, false));
  if (c.flags) {
    *done = 1;
    fill_reports(S, c, r, br);
    return fail(flag_code(c.flags), "slot faulted");
  }
  if (complete) {
    *done = 1;
    fill_reports(S, c, r, br);
  }
  return SPH_OK;
}

static int slot_get_fluid(sph_pool* P, SlotHost& S, double* x, double* v, double* rho, double* T);

extern "C" int sph_pool_get_fluid(sph_pool* P, int32_t slot, double* x, double* v, double* rho, double* T) {
  if (!P || slot < 0 || slot >= P->max_slots || !P->slots[slot].used) return fail(SPH_ERR_ARG, "bad slot");
  return slot_get_fluid(P, P->slots[slot], x, v, rho, T);
}

extern "C" int sph_pool_release(sph_pool* P, int32_t slot) {
  if (!P || slot < 0 || slot >= P->max_slots || !P->slots[slot].used) return fail(SPH_ERR_ARG, "bad slot");
  SlotHost& S = P->slots[slot];
  // Stream-ordered release: work already enqueued for this slot precedes any
  // later use of the memory on the same stream.  Launches from here on no
  // longer include the slot.
  P->comp_dirty = true;
  dev_free(P, S.arena);
  if (S.ev_done) (void)hipEventDestroy(S.ev_done);
  if (S.ev_admit) (void)hipEventDestroy(S.ev_admit);
  P->used -= S.bytes;
  S = SlotHost();
  return SPH_OK;
}

extern "C" int sph_pool_usage(sph_pool* P, size_t* bytes, int32_t* active) {
  if (!P) return fail(SPH_ERR_ARG, "NULL pool");
  if (bytes) *bytes = P->used;
  int a = 0;
  for (int s = 0; s < P->max_slots; ++s) a += P->slots[s].used ? 1 : 0;
  if (active) *active = a;
  return SPH_OK;
}

extern "C" int sph_pool_set_graph(sph_pool* P, int32_t enable) {
  if (!P) return fail(SPH_ERR_ARG, "NULL pool");
  P->use_graph = enable && P->stream != nullptr;
  drop_graph(P);
  return SPH_OK;
}

extern "C" int sph_pool_destroy(sph_pool* P) {
  if (!P) return SPH_OK;
  (void)hipStreamSynchronize(P->stream);
  drop_graph(P);
  for (int s = 0; s < MAX_SLOTS; ++s) {
    SlotHost& S = P->slots[s];
    if (S.used) {
      dev_free(P, S.arena);
      if (S.ev_done) (void)hipEventDestroy(S.ev_done);
      if (S.ev_admit) (void)hipEventDestroy(S.ev_admit);
    }
  }
  dev_free(P, P->d_table);
  for (auto& t : P->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : P->free_events) (void)hipEventDestroy(e);
  if (P->copy_stream) (void)hipStreamDestroy(P->copy_stream);
  if (P->side_stream) (void)hipStreamDestroy(P->side_stream);
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  if (P->ev_join) (void)hipEventDestroy(P->ev_join);
  delete P;
  return SPH_OK;
}

// ---------------------------------------------------------------------------
// read-back helpers
// ---------------------------------------------------------------------------
static int d2h(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return SPH_OK;
  HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  return SPH_OK;
}

static double get_as_double(const char* base, size_t idx, size_t sz) {
  if (sz == 8) {
    double d;
    std::memcpy(&d, base + idx * 8, 8);
    return d;
  }
  float f;
  std::memcpy(&f, base + idx * 4, 4);
  return (double)f;
}

static int slot_get_fluid(sph_pool* P, SlotHost& S, double* x, double* v, double* rho, double* T) {
  HIPCHK(hipStreamSynchronize(P->stream));
  const Plan& pl = S.plan;
  const size_t nf = (size_t)pl.nf;
  std::vector<uint32_t> fid(nf);
  std::vector<char> xa(4 * nf * pl.pos_sz), dr(4 * nf * pl.real_sz), vv(4 * nf * pl.real_sz), tt(nf * pl.temp_sz);
  LCHK(d2h(fid.data(), S.d.fid, nf * 4));
  LCHK(d2h(xa.data(), S.d.xa, xa.size()));
  LCHK(d2h(dr.data(), S.d.drift, dr.size()));
  LCHK(d2h(vv.data(), S.d.vr, vv.size()));
  LCHK(d2h(tt.data(), S.d.T, tt.size()));
  const bool rel = pl.prec != SPH_PREC_FP32;
  for (size_t k = 0; k < nf; ++k) {
    const size_t o = fid[k];
    for (size_t a = 0; a < 3; ++a) {
      if (x) x[3 * o + a] = get_as_double(xa.data(), 4 * k + a, pl.pos_sz) + get_as_double(dr.data(), 4 * k + a, pl.real_sz);
      if (v) v[3 * o + a] = get_as_double(vv.data(), 4 * k + a, pl.real_sz);
    }
    if (rho) rho[o] = get_as_double(vv.data(), 4 * k + 3, pl.real_sz) + (rel ? S.params.rho0 : 0.0);
    if (T) T[o] = get_as_double(tt.data(), k, pl.temp_sz);
  }
  return SPH_OK;
}

// ---------------------------------------------------------------------------
// single solver = pool with one slot
// ---------------------------------------------------------------------------
extern "C" int sph_create(const sph_params* p, const sph_allocator* a, void* stream, sph_solver** out) {
  if (!out) return fail(SPH_ERR_ARG, "out is NULL");
  *out = nullptr;
  Plan tmp;
  int rc = make_plan(p, p ? p->precision : 0, 1, 0, &tmp);
  if (rc) return rc;
  sph_solver* s = new sph_solver();
  s->p = *p;
  rc = sph_pool_create((size_t)-1, 1, p->precision, a, stream, &s->pool);
  if (rc) {
    delete s;
    return rc;
  }
  *out = s;
  return SPH_OK;
}

extern "C" int sph_set_bodies(sph_solver* s, int32_t n, const sph_body* b) {
  if (!s || !b || n < 1 || n > NB) return fail(SPH_ERR_ARG, "need 1..8 bodies");
  if (s->inited) return fail(SPH_ERR_STATE, "already initialised");
  s->nbody = n;
  for (int k = 0; k < n; ++k) s->bodies[k] = b[k];
  return SPH_OK;
}

extern "C" int sph_set_fluid(sph_solver* s, int64_t n, const double* x, const double* v, const double* rho,
                             const double* T, const int32_t* material) {
  if (!s || n < 1 || !x || !rho || !T) return fail(SPH_ERR_ARG, "fluid arrays missing");
  if (s->inited) return fail(SPH_ERR_STATE, "already initialised");
  s->nf = n;
  s->x.assign(x, x + 3 * n);
  s->v.assign((size_t)(3 * n), 0.0);
  if (v) s->v.assign(v, v + 3 * n);
  s->rho.assign(rho, rho + n);
  s->T.assign(T, T + n);
  s->material.clear();
  if (material) s->material.assign(material, material + n);
  return SPH_OK;
}

extern "C" int sph_set_solid(sph_solver* s, int64_t n, const double* x0, const double* n0, const int32_t* body) {
  if (!s || n < 0 || (n > 0 && (!x0 || !n0 || !body))) return fail(SPH_ERR_ARG, "solid arrays missing");
  if (s->inited) return fail(SPH_ERR_STATE, "already initialised");
  s->ns = n;
  s->x0.assign(x0, x0 + 3 * n);
  s->n0.assign(n0, n0 + 3 * n);
  s->body.assign(body, body + n);
  return SPH_OK;
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free contact factor: per-block, per-body partial
// sums (value and count) of at most SPH_CONTACT_NOALLOC_MAX_SOLID solid
// particles, 2 MiB.  Each GPU holds its own copy until the process ends;
// every call on a GPU shares it, so calls that overlap on one GPU race.  In
// host code `scratch` is only a host-side stand-in: the device address comes
// from hipGetSymbolAddress, once per device, and only that address is used.
// ---------------------------------------------------------------------------
constexpr int NOALLOC_MAX_BLOCKS = (int)(SPH_CONTACT_NOALLOC_MAX_SOLID / BLOCK);
static __device__ __align__(256) double scratch[2 * NB * NOALLOC_MAX_BLOCKS];
constexpr int MAX_DEVICES = 64;
static double* g_scratch[MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// the device address of `scratch` on the current device (looked up once)
static int scratch_address(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail_lit(SPH_ERR_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= MAX_DEVICES) return fail_lit(SPH_ERR_STATE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return fail_lit(SPH_ERR_HIP, "hipGetSymbolAddress(scratch) failed");
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return SPH_OK;
}

extern "C" int sph_init(sph_solver* s) {
  if (!s) return fail(SPH_ERR_ARG, "NULL solver");
  if (s->inited) return fail(SPH_ERR_STATE, "already initialised");
  if (s->nbody < 1 || s->nf < 1) return fail(SPH_ERR_STATE, "bodies and fluid must be set first");
  {
    double* scr = nullptr;   // set-up of the allocation-free entry point's scratch on this device
    LCHK(scratch_address(&scr));
  }
  int32_t slot = -1;
  int rc = admit(s->pool, &s->p, s->nbody, s->bodies, s->nf, s->x.data(), s->v.data(), s->rho.data(), s->T.data(),
                 s->material.empty() ? nullptr : s->material.data(), s->ns, s->x0.data(), s->n0.data(),
                 s->body.data(), INT64_MAX, &slot);
  if (rc) return rc;
  sph_pool* P = s->pool;
  LaunchTab T;
  tab_for(P, std::vector<int>{slot}, T);
  rc = enqueue_sort_build(P, T);
  if (rc) return rc;
  LCHK(launch(P, T, SPH_K_VISC_HEAT, 0, 0));   // frozen rates for the first step
  SlotCtl c;
  LCHK(read_ctl(P, P->slots[slot], &c, true));
  s->inited = true;
  s->x.clear();
  s->v.clear();
  s->rho.clear();
  s->T.clear();
  s->material.clear();
  if (c.flags) return fail(flag_code(c.flags), "initial build faulted");
  return SPH_OK;
}

extern "C" int sph_step(sph_solver* s, int32_t n) {
  if (!s || !s->inited) return fail(SPH_ERR_STATE, "not initialised");
  return pool_step(s->pool, n);
}

extern "C" int sph_reduce(sph_solver* s, sph_report* r, sph_body_report* br) {
  if (!s || !s->inited) return fail(SPH_ERR_STATE, "not initialised");
  SlotHost& S = s->pool->slots[0];
  SlotCtl c;
  LCHK(read_ctl(s->pool, S, &c, true));
  fill_reports(S, c, r, br);
  if (c.flags) return fail(flag_code(c.flags), "solve faulted");
  return SPH_OK;
}

extern "C" int sph_contact_factor(sph_solver* s, double* zeta, double* body_mean) {
  if (!s || !s->inited) return fail(SPH_ERR_STATE, "not initialised");
  sph_pool* P = s->pool;
  SlotHost& S = P->slots[0];
  SlotCtl c;
  LCHK(read_ctl(P, S, &c, true));
  if (c.flags) return fail(flag_code(c.flags), "solve faulted");
  LaunchTab T;
  tab_for(P, std::vector<int>{0}, T);
  LCHK(enqueue_sort_build(P, T, true, false));
  LCHK(launch(P, T, SPH_K_CONTACT, 1, 0));
  LCHK(read_ctl(P, S, &c, true));
  if (c.flags) return fail(flag_code(c.flags), "contact factor build faulted");
  const size_t ns = (size_t)S.plan.ns;
  // the kernel wrote the values in the original order: one read-back
  std::vector<double> tmp;
  double* z = zeta;
  if (!z && body_mean) {
    tmp.resize(ns);
    z = tmp.data();
  }
  if (z && ns) LCHK(d2h(z, S.d.zeta, ns * 8));
  if (body_mean) {
    // mean per body over its particles in their original order, compensated
    for (int b = 0; b < S.nbody; ++b) {
      double sum = 0.0, comp = 0.0;
      int64_t cnt = 0;
      for (size_t k = 0; k < ns; ++k) {
        if (s->body[k] != b) continue;
        const double t = sum + z[k];
        comp += std::fabs(sum) >= std::fabs(z[k]) ? (sum - t) + z[k] : (z[k] - t) + sum;
        sum = t;
        ++cnt;
      }
      body_mean[b] = cnt ? (sum + comp) / (double)cnt : 0.0;
    }
  }
  return SPH_OK;
}

extern "C" int sph_contact_factor_noalloc(sph_solver* s, double* zeta_dev, double* body_mean_dev) {
  if (!s || !s->inited) return fail_lit(SPH_ERR_STATE, "not initialised");
  sph_pool* P = s->pool;
  const SlotHost& S = P->slots[0];
  if (S.plan.ns > (int64_t)SPH_CONTACT_NOALLOC_MAX_SOLID)
    return fail_lit(SPH_ERR_ARG, "more solid particles than SPH_CONTACT_NOALLOC_MAX_SOLID");
  if (S.plan.nblk[DOM_SOLID] > NOALLOC_MAX_BLOCKS) return fail_lit(SPH_ERR_ARG, "solid blocks beyond the scratch");
  double* scr = nullptr;
  LCHK(scratch_address(&scr));
  LaunchTab T;
  tab_one(P, 0, T);
  LCHK(enqueue_sort_build(P, T, false, false));
  if (launch_contact(P->prec, P->d_table, T, zeta_dev, body_mean_dev ? scr : nullptr, body_mean_dev, P->stream) !=
      hipSuccess)
    return fail_lit(SPH_ERR_HIP, "contact factor launch failed");
  return SPH_OK;
}

static bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

extern "C" int sph_relax(sph_solver* s, const sph_shape* sh, int32_t iterations, sph_relax_report* rep) {
  if (!s || !s->inited) return fail(SPH_ERR_STATE, "not initialised");
  if (!sh) return fail(SPH_ERR_ARG, "shape is NULL");
  if (iterations < 1) return fail(SPH_ERR_ARG, "iterations must be >= 1");
  if (sh->inside != 0 && sh->inside != 1) return fail(SPH_ERR_ARG, "inside must be 0 or 1");
  if (sh->reserved != 0) return fail(SPH_ERR_ARG, "reserved must be 0");
  if (!finite3(sh->center) || !finite3(sh->size) || !std::isfinite(sh->phase))
    return fail(SPH_ERR_ARG, "non-finite shape");
  const double* z = sh->size;
  bool ok;
  switch (sh->kind) {
    case SPH_SHAPE_SPHERE: ok = z[0] > 0; break;
    case SPH_SHAPE_BOX: ok = z[0] > 0 && z[1] > 0 && z[2] > 0; break;
    case SPH_SHAPE_CYLINDER: ok = z[0] > 0 && z[1] > 0; break;
    case SPH_SHAPE_GEAR: ok = z[1] > 0 && z[0] > z[1] && z[2] > 0 && sh->teeth >= 2 && sh->teeth <= 512; break;
    default: return fail(SPH_ERR_ARG, "unknown shape kind");
  }
  if (!ok) return fail(SPH_ERR_ARG, "shape sizes out of range");
  sph_pool* P = s->pool;
  SlotHost& S = P->slots[0];
  SlotCtl c;
  LCHK(read_ctl(P, S, &c, true));
  if (c.flags) return fail(flag_code(c.flags), "solve faulted");
  RelaxShape g;
  g.kind = sh->kind;
  g.teeth = sh->teeth;
  g.inside = sh->inside;
  g.pad = 0;
  for (int a = 0; a < 3; ++a) {
    g.center[a] = sh->center[a];
    g.size[a] = sh->size[a];
  }
  g.phase = sh->phase - std::floor(sh->phase);   // the same teeth; keeps the tooth index small
  g.zu = (double)sh->teeth / (2.0 * M_PI);
  LaunchTab T;
  tab_for(P, std::vector<int>{0}, T);
  for (int it = 0; it < iterations; ++it) {
    LCHK(enqueue_sort_build(P, T, true, false));
    LCHK(launch_rx(P, T, SPH_K_RELAX_FORCE, it, g));
    LCHK(launch_rx(P, T, SPH_K_RELAX_MAX, it, g));
    LCHK(launch_rx(P, T, SPH_K_RELAX_MOVE, it, g));
  }
  LCHK(read_ctl(P, S, &c, true));
  if (c.flags) return fail(flag_code(c.flags), "relaxation faulted");
  if (rep) {
    rep->iterations = iterations;
    rep->bounded_last = c.relax_bounded;
    rep->amax_first = c.relax_first;
    rep->amax_last = c.relax_amax;
    rep->dt_last = c.relax_dt;
  }
  return SPH_OK;
}

extern "C" int sph_get_fluid(sph_solver* s, double* x, double* v, double* rho, double* T) {
  if (!s || !s->inited) return fail(SPH_ERR_STATE, "not initialised");
  return slot_get_fluid(s->pool, s->pool->slots[0], x, v, rho, T);
}

extern "C" int sph_set_graph(sph_solver* s, int32_t enable) {
  if (!s) return fail(SPH_ERR_ARG, "NULL solver");
  return sph_pool_set_graph(s->pool, enable);
}

extern "C" int sph_set_timing(sph_solver* s, int32_t enable) {
  if (!s) return fail(SPH_ERR_ARG, "NULL solver");
  LCHK(collect_timing(s->pool));
  s->pool->timing = enable != 0;
  for (auto& t : s->pool->times) t.clear();
  return SPH_OK;
}

extern "C" int sph_get_timing(sph_solver* s, int32_t kid, int32_t max, float* ms, int32_t* count) {
  if (!s || kid < 0 || kid >= SPH_K_COUNT) return fail(SPH_ERR_ARG, "bad kernel id");
  LCHK(collect_timing(s->pool));
  const std::vector<float>& t = s->pool->times[kid];
  if (count) *count = (int32_t)t.size();
  if (ms)
    for (int32_t k = 0; k < max && k < (int32_t)t.size(); ++k) ms[k] = t[(size_t)k];
  return SPH_OK;
}

static size_t dump_bytes(const SlotHost& S, int what) {
  const Plan& pl = S.plan;
  const size_t nf = (size_t)pl.nf, ns = (size_t)pl.ns;
  switch (what) {
    case SPH_DUMP_FLUID_IDS: return nf * 4;
    case SPH_DUMP_SOLID_IDS: return ns * 4;
    case SPH_DUMP_FLUID_CELL: return nf * 4;
    case SPH_DUMP_NBR_COUNT: return 2 * nf * 4;
    case SPH_DUMP_NBR_FLUID: return nf * (size_t)pl.kf * 4;
    case SPH_DUMP_NBR_SOLID: return nf * (size_t)pl.ks * 4;
    case SPH_DUMP_FLUID_OFFSET: return nf * 4 * 8;
    case SPH_DUMP_SOLID_OFFSET: return ns * 4 * 8;
    case SPH_DUMP_FLUID_STATE: return nf * 16 * 8;
    case SPH_DUMP_SOLID_STATE: return ns * 13 * 8;
    case SPH_DUMP_SUMW: return nf * 8;
    case SPH_DUMP_SOLID_DUMMY: return ns * 4 * 8;
    default: return 0;
  }
}

extern "C" int sph_dump_size(sph_solver* s, int32_t what, size_t* bytes) {
  if (!s || !s->inited || !bytes) return fail(SPH_ERR_STATE, "not initialised");
  *bytes = dump_bytes(s->pool->slots[0], what);
  return *bytes ? SPH_OK : fail(SPH_ERR_ARG, "unknown dump selector");
}

// rows of SELL storage [slice][k][lane] -> [particle][k]
template <class F>
static void unsell(const Plan& pl, int K, F&& f) {
  const size_t nf = (size_t)pl.nf;
  for (size_t i = 0; i < nf; ++i) {
    const size_t sl = i / WAVE, ln = i % WAVE;
    for (int k = 0; k < K; ++k) f(i, k, (sl * (size_t)K + (size_t)k) * WAVE + ln);
  }
}

extern "C" int sph_debug_dump(sph_solver* s, int32_t what, void* buf, size_t bytes) {
  if (!s || !s->inited || !buf) return fail(SPH_ERR_STATE, "not initialised");
  SlotHost& S = s->pool->slots[0];
  const size_t need = dump_bytes(S, what);
  if (!need) return fail(SPH_ERR_ARG, "unknown dump selector");
  if (bytes < need) return fail(SPH_ERR_ARG, "buffer too small");
  HIPCHK(hipStreamSynchronize(s->pool->stream));
  const Plan& pl = S.plan;
  const SlotDesc& D = S.d;
  const size_t nf = (size_t)pl.nf, ns = (size_t)pl.ns;
  const size_t rs = pl.real_sz, ps = pl.pos_sz, ts = pl.temp_sz;
  switch (what) {
    case SPH_DUMP_FLUID_IDS: return d2h(buf, D.fid, nf * 4);
    case SPH_DUMP_SOLID_IDS: return d2h(buf, D.sid, ns * 4);
    case SPH_DUMP_FLUID_CELL: {
      // the cell of sorted particle k is the run [start[r], start[r+1]) holding k
      std::vector<uint32_t> st((size_t)pl.ncells + 1);
      LCHK(d2h(st.data(), D.start_f, st.size() * 4));
      uint32_t* o = (uint32_t*)buf;
      for (size_t i = 0; i < nf; ++i) {
        const size_t r = (size_t)(std::upper_bound(st.begin(), st.end(), (uint32_t)i) - st.begin()) - 1;
        o[i] = S.morton_of_rank[r];
      }
      return SPH_OK;
    }
    case SPH_DUMP_NBR_COUNT: {
      LCHK(d2h(buf, D.nfc, nf * 4));
      return d2h((char*)buf + nf * 4, D.nsc, nf * 4);
    }
    case SPH_DUMP_NBR_FLUID:
    case SPH_DUMP_NBR_SOLID: {
      const bool sol = what == SPH_DUMP_NBR_SOLID;
      const int K = sol ? pl.ks : pl.kf;
      const size_t L = (size_t)(sol ? pl.rowlen_s : pl.rowlen_f);
      std::vector<uint32_t> r(L);
      LCHK(d2h(r.data(), sol ? D.srec : D.nrec, r.size() * 4));
      uint32_t* o = (uint32_t*)buf;
      unsell(pl, K, [&](size_t i, int k, size_t src) { o[i * (size_t)K + (size_t)k] = r[src]; });
      return SPH_OK;
    }
    case SPH_DUMP_FLUID_OFFSET:
    case SPH_DUMP_SOLID_OFFSET: {
      // (ox, oy, oz) as stored, then the packed cell coordinates as a number
      const bool sol = what == SPH_DUMP_SOLID_OFFSET;
      const size_t n = sol ? ns : nf;
      std::vector<char> r(4 * n * rs);
      LCHK(d2h(r.data(), sol ? D.so : D.xo, r.size()));
      double* o = (double*)buf;
      for (size_t i = 0; i < n; ++i) {
        for (size_t a = 0; a < 3; ++a) o[4 * i + a] = get_as_double(r.data(), 4 * i + a, rs);
        uint32_t c;
        if (rs == 8) {
          double d;
          std::memcpy(&d, r.data() + (4 * i + 3) * 8, 8);
          c = (uint32_t)d;
        } else {
          std::memcpy(&c, r.data() + (4 * i + 3) * 4, 4);
        }
        o[4 * i + 3] = (double)c;
      }
      return SPH_OK;
    }
    case SPH_DUMP_FLUID_STATE: {
      std::vector<char> xa(4 * nf * ps), dr(4 * nf * rs), v(4 * nf * rs), drho(nf * rs), T(nf * ts), ah(4 * nf * rs);
      LCHK(d2h(xa.data(), D.xa, xa.size()));
      LCHK(d2h(dr.data(), D.drift, dr.size()));
      LCHK(d2h(v.data(), D.vr, v.size()));
      LCHK(d2h(drho.data(), D.drho, drho.size()));
      LCHK(d2h(T.data(), D.T, T.size()));
      LCHK(d2h(ah.data(), D.ah, ah.size()));
      const bool rel = pl.prec != SPH_PREC_FP32;
      double* o = (double*)buf;
      for (size_t i = 0; i < nf; ++i) {
        double* e = o + i * 16;
        for (size_t a = 0; a < 3; ++a) {
          e[a] = get_as_double(xa.data(), 4 * i + a, ps);
          e[3 + a] = get_as_double(dr.data(), 4 * i + a, rs);
          e[6 + a] = get_as_double(v.data(), 4 * i + a, rs);
          e[12 + a] = get_as_double(ah.data(), 4 * i + a, rs);
        }
        e[9] = get_as_double(v.data(), 4 * i + 3, rs) + (rel ? S.params.rho0 : 0.0);
        e[10] = get_as_double(drho.data(), i, rs);
        e[11] = get_as_double(T.data(), i, ts);
        e[15] = get_as_double(ah.data(), 4 * i + 3, rs);
      }
      return SPH_OK;
    }
    case SPH_DUMP_SOLID_STATE: {
      std::vector<char> x(4 * ns * ps), n(4 * ns * rs), v(4 * ns * rs), l(4 * ns * rs);
      std::vector<int32_t> b(ns);
      LCHK(d2h(x.data(), D.xw, x.size()));
      LCHK(d2h(n.data(), D.nw, n.size()));
      LCHK(d2h(v.data(), D.vw, v.size()));
      LCHK(d2h(l.data(), D.lev, l.size()));
      LCHK(d2h(b.data(), D.body, ns * 4));
      double* o = (double*)buf;
      for (size_t w = 0; w < ns; ++w) {
        double* e = o + w * 13;
        for (size_t a = 0; a < 3; ++a) {
          e[a] = get_as_double(x.data(), 4 * w + a, ps);
          e[3 + a] = get_as_double(n.data(), 4 * w + a, rs);
          e[6 + a] = get_as_double(v.data(), 4 * w + a, rs);
          e[9 + a] = get_as_double(l.data(), 4 * w + a, rs);
        }
        e[12] = (double)b[w];
      }
      return SPH_OK;
    }
    case SPH_DUMP_SUMW: return d2h(buf, D.sumW, nf * 8);
    case SPH_DUMP_SOLID_DUMMY: {
      std::vector<char> r(4 * ns * rs);
      LCHK(d2h(r.data(), D.vd, r.size()));
      double* o = (double*)buf;
      for (size_t k = 0; k < 4 * ns; ++k) o[k] = get_as_double(r.data(), k, rs);
      return SPH_OK;
    }
    default: return fail(SPH_ERR_ARG, "unknown dump selector");
  }
}

extern "C" int sph_debug_set_fusion(sph_solver* s, int32_t enable) {
  if (!s) return fail(SPH_ERR_ARG, "NULL solver");
  if (enable != 0 && enable != 1) return fail(SPH_ERR_ARG, "enable must be 0 or 1");
  s->pool->fuse_first = enable == 1;
  drop_graph(s->pool);
  return SPH_OK;
}

extern "C" int sph_debug_poke_velocity(sph_solver* s, int64_t orig, const double* v3) {
  if (!s || !s->inited || !v3) return fail(SPH_ERR_STATE, "not initialised");
  SlotHost& S = s->pool->slots[0];
  const Plan& pl = S.plan;
  if (orig < 0 || orig >= pl.nf) return fail(SPH_ERR_ARG, "index out of range");
  HIPCHK(hipStreamSynchronize(s->pool->stream));
  std::vector<uint32_t> fid((size_t)pl.nf);
  LCHK(d2h(fid.data(), S.d.fid, fid.size() * 4));
  size_t k = 0;
  while (k < fid.size() && fid[k] != (uint32_t)orig) ++k;
  if (k == fid.size()) return fail(SPH_ERR_ARG, "index not found");
  for (size_t a = 0; a < 3; ++a) {
    char* dst = (char*)S.d.vr + (4 * k + a) * pl.real_sz;
    if (pl.real_sz == 8) {
      HIPCHK(hipMemcpy(dst, &v3[a], 8, hipMemcpyHostToDevice));
    } else {
      const float f = (float)v3[a];
      HIPCHK(hipMemcpy(dst, &f, 4, hipMemcpyHostToDevice));
    }
  }
  return SPH_OK;
}

extern "C" int sph_destroy(sph_solver* s) {
  if (!s) return SPH_OK;
  int rc = sph_pool_destroy(s->pool);
  delete s;
  return rc;
}
