"""ctypes wrapper of the FP64 CPU oracle (sph_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sph_oracle.c")
LIB = os.path.join(HERE, "libsph_oracle.so")

ORA_OK, ORA_ERR_ARG, ORA_ERR_OOM, ORA_ERR_DOMAIN = 0, 1, 2, 5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def set_threads(n: int) -> int:
    """Set the OpenMP thread count of the oracle's later calls from this
    thread; returns the previous count."""
    lib()
    gomp = C.CDLL("libgomp.so.1")
    prev = int(gomp.omp_get_max_threads())
    gomp.omp_set_num_threads(C.c_int(int(n)))
    return prev


class Params(C.Structure):
    _fields_ = [("dp", C.c_double), ("h_over_dp", C.c_double), ("rho0", C.c_double),
                ("c0", C.c_double), ("nu", C.c_double), ("k_f", C.c_double), ("cp_f", C.c_double),
                ("gravity", C.c_double * 3), ("grid_lo", C.c_double * 3), ("grid_hi", C.c_double * 3),
                ("cfl_ad", C.c_double), ("cfl_ac", C.c_double), ("fixed_dt_ad", C.c_double),
                ("fixed_nac", C.c_int32), ("nac_max", C.c_int32), ("free_surface", C.c_int32),
                ("eq13_printed", C.c_int32), ("viscous_heating", C.c_int32), ("wall_visc", C.c_int32)]


class BodyS(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("axis", C.c_double * 3), ("omega", C.c_double),
                ("T", C.c_double), ("k", C.c_double)]


class Report(C.Structure):
    _fields_ = [("t", C.c_double), ("dt_ad", C.c_double), ("dt", C.c_double), ("n_ac", C.c_int32),
                ("pad", C.c_int32), ("vmax", C.c_double), ("mass", C.c_double),
                ("kinetic", C.c_double), ("thermal", C.c_double), ("heat_step", C.c_double),
                ("mass_proxy", C.c_double), ("diss_step", C.c_double)]


class BodyReport(C.Structure):
    _fields_ = [("force", C.c_double * 3), ("torque", C.c_double * 3), ("torque_axis", C.c_double),
                ("power", C.c_double), ("heat_rate", C.c_double)]


class Rates(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("a_visc", "dTdt", "sumW", "S_visc", "S_T", "a_p", "S_p", "S_rho",
                                          "G", "phi", "S_G", "bscale")]


_lib = None
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.ora_kernel_W.restype = C.c_double
        L.ora_kernel_W.argtypes = [C.c_double, C.c_double]
        L.ora_kernel_dW.restype = C.c_double
        L.ora_kernel_dW.argtypes = [C.c_double, C.c_double]
        L.ora_kernel_F.restype = C.c_double
        L.ora_kernel_F.argtypes = [C.c_double, C.c_double]
        L.ora_lattice_sum0.restype = C.c_double
        L.ora_lattice_sum0.argtypes = [C.c_double]
        L.ora_lattice_halfspace.restype = C.c_double
        L.ora_lattice_halfspace.argtypes = [C.c_double]
        L.ora_morton3.restype = C.c_uint32
        L.ora_morton3.argtypes = [C.c_uint32] * 3
        L.ora_nbr_total.restype = C.c_int64
        L.ora_nbr_total.argtypes = [C.c_void_p, C.c_int32]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_params(params: dict, **over) -> Params:
    d = dict(params)
    d.update(over)
    P = Params()
    for k in ("dp", "h_over_dp", "rho0", "c0", "nu", "k_f", "cp_f", "cfl_ad", "cfl_ac", "fixed_dt_ad"):
        setattr(P, k, float(d.get(k, 0.0)))
    for k in ("gravity", "grid_lo", "grid_hi"):
        getattr(P, k)[:] = [float(v) for v in d[k]]
    P.fixed_nac = int(d.get("fixed_nac", 0))
    P.nac_max = int(d.get("nac_max", 16))
    P.free_surface = int(d.get("free_surface", 1))
    P.eq13_printed = int(d.get("eq13_printed", 0))
    P.viscous_heating = int(d.get("viscous_heating", 0))
    P.wall_visc = int(d.get("wall_visc", 0))   # 0: Shepard no-slip dummy velocity
    return P


def make_bodies(bodies) -> C.Array:
    arr = (BodyS * max(1, len(bodies)))()
    for i, b in enumerate(bodies):
        d = b.as_dict() if hasattr(b, "as_dict") else b
        arr[i].center[:] = list(d["center"])
        arr[i].axis[:] = list(d["axis"])
        arr[i].omega = d["omega"]
        arr[i].T = d["T"]
        arr[i].k = d["k"]
    return arr


def W(r, h):
    return lib().ora_kernel_W(float(r), float(h))


def dW(r, h):
    return lib().ora_kernel_dW(float(r), float(h))


def F(r, h):
    return lib().ora_kernel_F(float(r), float(h))


def lattice_sum0(h_over_dp):
    return lib().ora_lattice_sum0(float(h_over_dp))


def lattice_halfspace(h_over_dp):
    """Kernel sum (units of dp^3) over the lattice half-space x > 0: the
    full-immersion reference of the contact factor (eq. 24)."""
    return lib().ora_lattice_halfspace(float(h_over_dp))


def contact_factor(params, xf, rho, xs, ref=None):
    """Contact factor of every solid particle at positions xs (eq. 24)."""
    P = make_params(params)
    xf = _c3(xf)
    xs = _c3(xs)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    if ref is None:
        ref = lattice_halfspace(params["h_over_dp"])
    z = np.zeros(len(xs))
    rc = lib().ora_contact_factor(C.byref(P), C.c_int64(len(xf)), _p(xf), _p(rho), C.c_int64(len(xs)), _p(xs),
                                  C.c_double(ref), _p(z))
    if rc != 0:
        raise RuntimeError(f"ora_contact_factor failed: {rc}")
    return z


def morton3(cx, cy, cz):
    return int(lib().ora_morton3(cx, cy, cz))


def _c3(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3))


def cells(params: dict, x):
    x = _c3(x)
    out = np.zeros((len(x), 3), dtype=np.int32)
    rc = lib().ora_cells(C.byref(make_params(params)), C.c_int64(len(x)), _p(x), _p(out))
    return rc, out


def grid_dims(params: dict):
    d = (C.c_int32 * 3)()
    rc = lib().ora_grid_dims(C.byref(make_params(params)), d)
    return rc, tuple(d)


def sort_order(params: dict, x, ids=None):
    x = _c3(x)
    if ids is None:
        ids = np.arange(len(x), dtype=np.uint32)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    order = np.zeros(len(x), dtype=np.int64)
    rc = lib().ora_sort_order(C.byref(make_params(params)), C.c_int64(len(x)), _p(x), _p(ids), _p(order))
    return rc, order


class Nbr:
    """Neighbour sets (fluid and solid) with the frozen geometry of a build."""

    def __init__(self, params: dict, xf, xs=None, brute=False):
        self.P = make_params(params)
        self.xf = _c3(xf)
        self.xs = _c3(np.zeros((0, 3)) if xs is None else xs)
        h = C.c_void_p()
        rc = lib().ora_nbr_build(C.byref(self.P), C.c_int64(len(self.xf)), _p(self.xf),
                                 C.c_int64(len(self.xs)), _p(self.xs), C.c_int32(int(brute)), C.byref(h))
        if rc != 0:
            raise RuntimeError(f"ora_nbr_build failed: {rc}")
        self.h = h

    def csr(self, which=0):
        n = len(self.xf)
        tot = lib().ora_nbr_total(self.h, which)
        off = np.zeros(n + 1, dtype=np.int64)
        idx = np.zeros(max(tot, 1), dtype=np.int32)
        lib().ora_nbr_csr(self.h, C.c_int32(which), _p(off), _p(idx))
        return off, idx[:tot]

    def sets(self, which=0):
        off, idx = self.csr(which)
        return [frozenset(idx[off[i]:off[i + 1]].tolist()) for i in range(len(off) - 1)]

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ora_nbr_free(self.h)
                self.h = None
        except Exception:
            pass


def sum_w(params, nbr: Nbr):
    out = np.zeros(len(nbr.xf))
    lib().ora_sum_w(C.byref(nbr.P), nbr.h, _p(out))
    return out


def _bodies_arg(bodies):
    if not bodies:
        return 0, None
    return len(bodies), make_bodies(bodies)


def viscous(params, nbr: Nbr, v, rho, mass, vs=None, bodies=(), body=None):
    nb, B = _bodies_arg(bodies)
    n = len(nbr.xf)
    v = _c3(v)
    vs = _c3(np.zeros((len(nbr.xs), 3)) if vs is None else vs)
    body = np.ascontiguousarray(np.zeros(len(nbr.xs), np.int32) if body is None else body, dtype=np.int32)
    a = np.zeros((n, 3))
    S = np.zeros(n)
    bF = np.zeros((max(nb, 1), 3))
    bT = np.zeros((max(nb, 1), 3))
    lib().ora_viscous(C.byref(nbr.P), nbr.h, C.c_int32(nb), B, _p(body), _p(v),
                      _p(np.ascontiguousarray(rho, dtype=np.float64)),
                      _p(np.ascontiguousarray(mass, dtype=np.float64)), _p(vs), _p(a), _p(S),
                      _p(bF) if nb else None, _p(bT) if nb else None)
    return a, S, bF[:nb], bT[:nb]


def wall_dummy_velocity(params, nbr: Nbr, v, vs):
    """Dummy velocity of every solid particle in the wall viscous force (eq. 18)
    under params["wall_visc"], and its Shepard weight sum."""
    ns = len(nbr.xs)
    vd = np.zeros((ns, 3))
    sw = np.zeros(ns)
    lib().ora_wall_dummy_velocity(C.byref(nbr.P), nbr.h, _p(_c3(v)), _p(_c3(vs)), _p(vd), _p(sw))
    return vd, sw


def heat(params, nbr: Nbr, rho, mass, k, cp, T, bodies=(), body=None):
    nb, B = _bodies_arg(bodies)
    n = len(nbr.xf)
    body = np.ascontiguousarray(np.zeros(len(nbr.xs), np.int32) if body is None else body, dtype=np.int32)
    out = np.zeros(n)
    S = np.zeros(n)
    bq = np.zeros(max(nb, 1))
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    lib().ora_heat(C.byref(nbr.P), nbr.h, C.c_int32(nb), B, _p(body), _p(f64(rho)), _p(f64(mass)),
                   _p(f64(k)), _p(f64(cp)), _p(f64(T)), _p(out), _p(S), _p(bq) if nb else None)
    return out, S, bq[:nb]


def velocity_gradient(params, nbr: Nbr, v, rho, mass, vs=None):
    """Velocity gradient G[i, a, b] = d v_a / d x_b (SPH gradient over fluid and
    wall neighbours) and the per-particle sum of |pair terms|."""
    n = len(nbr.xf)
    vs = _c3(np.zeros((len(nbr.xs), 3)) if vs is None else vs)
    G = np.zeros((n, 3, 3))
    S = np.zeros(n)
    f64 = lambda a_: np.ascontiguousarray(a_, dtype=np.float64)
    lib().ora_velocity_gradient(C.byref(nbr.P), nbr.h, _p(_c3(v)), _p(f64(rho)), _p(f64(mass)), _p(vs),
                                _p(G), _p(S))
    return G, S


def dissipation(params, G):
    """Viscous dissipation Phi = 2 eta S:S per particle (eq. 23)."""
    G = np.ascontiguousarray(G, dtype=np.float64).reshape(-1, 3, 3)
    out = np.zeros(len(G))
    lib().ora_dissipation(C.byref(make_params(params)), C.c_int64(len(G)), _p(G), _p(out))
    return out


def momentum(params, nbr: Nbr, v, rho, mass, nsv=None, vs=None, bodies=(), body=None):
    nb, B = _bodies_arg(bodies)
    n = len(nbr.xf)
    ns = len(nbr.xs)
    body = np.ascontiguousarray(np.zeros(ns, np.int32) if body is None else body, dtype=np.int32)
    nsv = _c3(np.zeros((ns, 3)) if nsv is None else nsv)
    vs = _c3(np.zeros((ns, 3)) if vs is None else vs)
    a = np.zeros((n, 3))
    S = np.zeros(n)
    bF = np.zeros((max(nb, 1), 3))
    bT = np.zeros((max(nb, 1), 3))
    f64 = lambda a_: np.ascontiguousarray(a_, dtype=np.float64)
    lib().ora_momentum(C.byref(nbr.P), nbr.h, C.c_int32(nb), B, _p(body), _p(_c3(v)), _p(f64(rho)),
                       _p(f64(mass)), _p(nsv), _p(vs), _p(a), _p(S),
                       _p(bF) if nb else None, _p(bT) if nb else None)
    return a, S, bF[:nb], bT[:nb]


def continuity(params, nbr: Nbr, v, rho, mass, nsv=None, vs=None):
    n = len(nbr.xf)
    ns = len(nbr.xs)
    nsv = _c3(np.zeros((ns, 3)) if nsv is None else nsv)
    vs = _c3(np.zeros((ns, 3)) if vs is None else vs)
    out = np.zeros(n)
    S = np.zeros(n)
    f64 = lambda a_: np.ascontiguousarray(a_, dtype=np.float64)
    lib().ora_continuity(C.byref(nbr.P), nbr.h, _p(_c3(v)), _p(f64(rho)), _p(f64(mass)), _p(nsv),
                         _p(vs), _p(out), _p(S))
    return out, S


def pair_force(params, xi, xj, vi, vj, rhoi, rhoj, mi, mj):
    f = np.zeros(6)
    f64 = lambda a_: np.ascontiguousarray(a_, dtype=np.float64)
    lib().ora_pair_force(C.byref(make_params(params)), _p(f64(xi)), _p(f64(xj)), _p(f64(vi)),
                         _p(f64(vj)), C.c_double(rhoi), C.c_double(rhoj), C.c_double(mi),
                         C.c_double(mj), _p(f))
    return f[:3].copy(), f[3:].copy()


def body_pose(bodies, x0, n0, body, t):
    nb, B = _bodies_arg(bodies)
    x0 = _c3(x0)
    n0 = _c3(n0)
    ns = len(x0)
    xs = np.zeros((ns, 3))
    nsv = np.zeros((ns, 3))
    vs = np.zeros((ns, 3))
    lib().ora_body_pose(C.c_int32(nb), B, C.c_int64(ns), _p(x0), _p(n0),
                        _p(np.ascontiguousarray(body, dtype=np.int32)), C.c_double(t), _p(xs), _p(nsv), _p(vs))
    return xs, nsv, vs


def totals(params, v, rho, T, cp=None):
    """Report totals of a fluid state: mass, kinetic energy, thermal energy,
    mass proxy sum rho dp^3, max |v| (compensated sums)."""
    out = np.zeros(5)
    f64 = lambda a_: np.ascontiguousarray(a_, dtype=np.float64)
    lib().ora_totals_cp(C.byref(make_params(params)), C.c_int64(len(rho)), _p(_c3(v)), _p(f64(rho)), _p(f64(T)),
                        _p(f64(cp)) if cp is not None else None, _p(out))
    return dict(mass=out[0], kinetic=out[1], thermal=out[2], mass_proxy=out[3], vmax=out[4])


def timestep(params, bodies, x0, body, v):
    nb, B = _bodies_arg(bodies)
    x0 = _c3(x0)
    v = _c3(v)
    dt_ad, dt, vmax = C.c_double(), C.c_double(), C.c_double()
    n_ac = C.c_int32()
    lib().ora_timestep(C.byref(make_params(params)), C.c_int32(nb), B, C.c_int64(len(x0)), _p(x0),
                       _p(np.ascontiguousarray(body, dtype=np.int32)), C.c_int64(len(v)), _p(v),
                       C.byref(dt_ad), C.byref(dt), C.byref(n_ac), C.byref(vmax))
    return dict(dt_ad=dt_ad.value, dt=dt.value, n_ac=n_ac.value, vmax=vmax.value)


class State:
    """Oracle state of one case: FP64 fluid arrays in the case's particle order."""

    def __init__(self, case, k=None, cp=None, **param_over):
        """k, cp: optional per-particle thermal conductivity and specific heat
        (several fluid materials); default the case's k_f, cp_f."""
        self.params = dict(case.params)
        self.params.update(param_over)
        self.k = None if k is None else np.ascontiguousarray(k, dtype=np.float64)
        self.cp = None if cp is None else np.ascontiguousarray(cp, dtype=np.float64)
        self.P = make_params(self.params)
        self.bodies = list(case.bodies)
        self.nb, self.B = _bodies_arg(self.bodies)
        self.x = case.xf.copy()
        self.v = case.vf.copy()
        self.rho = case.rhof.copy()
        self.T = case.Tf.copy()
        self.drho = np.zeros(case.nf)
        self.x0 = _c3(case.xs0)
        self.n0 = _c3(case.ns0)
        self.body = np.ascontiguousarray(case.body, dtype=np.int32)
        self.t = 0.0
        self.nstep = 0
        self.cum = dict(heat=0.0, torque_axis=np.zeros(self.nb), energy=np.zeros(self.nb))

    def step(self, want_rates=False):
        rep = Report()
        brep = (BodyReport * max(1, self.nb))()
        nf = len(self.x)
        rates = None
        rates_np = {}
        if want_rates:
            rates = Rates()
            for name, shape in (("a_visc", (nf, 3)), ("dTdt", (nf,)), ("sumW", (nf,)), ("S_visc", (nf,)),
                                ("S_T", (nf,)), ("a_p", (nf, 3)), ("S_p", (nf,)), ("S_rho", (nf,)),
                                ("G", (nf, 3, 3)), ("phi", (nf,)), ("S_G", (nf,)),
                                ("bscale", (max(1, self.nb), 13))):
                arr = np.zeros(shape)
                rates_np[name] = arr
                setattr(rates, name, arr.ctypes.data)
        t = C.c_double(self.t)
        rc = lib().ora_step_kc(C.byref(self.P), C.c_int32(self.nb), self.B, C.c_int64(nf), _p(self.x),
                               _p(self.v), _p(self.rho), _p(self.T), _p(self.drho), C.c_int64(len(self.x0)),
                               _p(self.x0), _p(self.n0), _p(self.body),
                               _p(self.k) if self.k is not None else None,
                               _p(self.cp) if self.cp is not None else None, C.byref(t), C.byref(rep), brep,
                               C.byref(rates) if rates is not None else None)
        if rc != 0:
            raise RuntimeError(f"ora_step failed: {rc}")
        self.t = t.value
        self.nstep += 1
        r = {k: getattr(rep, k) for k, _ in Report._fields_ if k != "pad"}
        bodies = []
        for b in range(self.nb):
            br = brep[b]
            bodies.append(dict(force=np.array(br.force[:]), torque=np.array(br.torque[:]),
                               torque_axis=br.torque_axis, power=br.power, heat_rate=br.heat_rate))
            self.cum["torque_axis"][b] += r["dt_ad"] * br.torque_axis
            self.cum["energy"][b] += r["dt_ad"] * br.power
        self.cum["heat"] += r["heat_step"]
        r["bodies"] = bodies
        if want_rates:
            r["rates"] = rates_np
        return r

    def totals(self):
        out = np.zeros(5)
        lib().ora_totals_cp(C.byref(self.P), C.c_int64(len(self.x)), _p(self.v), _p(self.rho), _p(self.T),
                            _p(self.cp) if self.cp is not None else None, _p(out))
        return dict(mass=out[0], kinetic=out[1], thermal=out[2], mass_proxy=out[3], vmax=out[4])


# ---------------------------------------------------------------------------
# physics-driven particle relaxation (Section 2.2, eq. 5-9)
# ---------------------------------------------------------------------------

SHAPES = {"sphere": 1, "box": 2, "cylinder": 3, "gear": 4}


class Shape(C.Structure):
    _fields_ = [("kind", C.c_int32), ("teeth", C.c_int32), ("inside", C.c_int32), ("pad", C.c_int32),
                ("center", C.c_double * 3), ("size", C.c_double * 3), ("phase", C.c_double)]


def make_shape(d: dict) -> Shape:
    """d: kind (sphere/box/cylinder/gear), center, size (3), teeth, phase, inside."""
    s = Shape()
    s.kind = SHAPES[d["kind"]]
    s.teeth = int(d.get("teeth", 0))
    s.inside = int(d.get("inside", 1))
    s.center[:] = [float(v) for v in d["center"]]
    sz = list(d["size"]) + [0.0] * (3 - len(d["size"]))
    s.size[:] = [float(v) for v in sz]
    s.phase = float(d.get("phase", 0.0))
    return s


def shape_phi(shape: dict, x):
    x = _c3(x)
    out = np.zeros(len(x))
    lib().ora_shape_eval(C.byref(make_shape(shape)), C.c_double(0.0), C.c_int64(len(x)), _p(x), _p(out), None)
    return out


def shape_normal(shape: dict, x, eps):
    x = _c3(x)
    out = np.zeros((len(x), 3))
    lib().ora_shape_eval(C.byref(make_shape(shape)), C.c_double(eps), C.c_int64(len(x)), _p(x), None, _p(out))
    return out


def exterior_integral(params, shape: dict, x):
    x = _c3(x)
    out = np.zeros((len(x), 3))
    lib().ora_exterior_integral_n(C.byref(make_params(params)), C.byref(make_shape(shape)), C.c_int64(len(x)),
                                  _p(x), _p(out))
    return out


def relax_step(params, shape: dict, x):
    """One relaxation iteration; returns (new positions, F_p, stats dict)."""
    x = _c3(x).copy()
    acc = np.zeros_like(x)
    st = np.zeros(3)
    rc = lib().ora_relax_step(C.byref(make_params(params)), C.byref(make_shape(shape)), C.c_int64(len(x)),
                              _p(x), _p(acc), _p(st))
    if rc != 0:
        raise RuntimeError(f"ora_relax_step failed: {rc}")
    return x, acc, dict(amax=st[0], dt=st[1], bounded=int(st[2]))
