"""Python binding of the C ABI in include/sph.h (argument marshalling only).

Every step of the hot path runs in the HIP library libsph.so; this module
only converts arrays, routes device allocations to PyTorch's caching
allocator and passes PyTorch's stream.  It fails loudly if the library has
not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

SPH_OK, SPH_ERR_ARG, SPH_ERR_OOM, SPH_ERR_HIP, SPH_ERR_STATE = 0, 1, 2, 3, 4
SPH_ERR_DOMAIN, SPH_ERR_NONFINITE, SPH_ERR_CAPACITY, SPH_ERR_BUDGET = 5, 6, 7, 8
PREC = {"mixed": 0, "fp64": 1, "fp32": 2}
MAX_BODIES = 8

KERNELS = ["clear", "pose", "fold", "scan1", "scan2", "scan3", "scatter", "cellsort", "reorder", "build",
           "dt", "visc_heat", "half_a", "momentum", "continuity", "end", "final", "sumw", "contact",
           "relax_force", "relax_max", "relax_move", "wallvel"]
K = {n: i for i, n in enumerate(KERNELS)}

DUMP = dict(fluid_ids=1, solid_ids=2, fluid_cell=3, nbr_count=4, nbr_fluid=5, nbr_solid=6, fluid_offset=7,
            solid_offset=8, fluid_state=9, solid_state=10, sumw=11, solid_dummy=12)


class SphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Params(C.Structure):
    _fields_ = [("dp", C.c_double), ("h_over_dp", C.c_double), ("rho0", C.c_double), ("c0", C.c_double),
                ("nu", C.c_double), ("k_f", C.c_double), ("cp_f", C.c_double), ("gravity", C.c_double * 3),
                ("grid_lo", C.c_double * 3), ("grid_hi", C.c_double * 3), ("cfl_ad", C.c_double),
                ("cfl_ac", C.c_double), ("fixed_dt_ad", C.c_double), ("fixed_nac", C.c_int32),
                ("nac_max", C.c_int32), ("free_surface", C.c_int32), ("precision", C.c_int32),
                ("max_fluid_nbrs", C.c_int32), ("max_solid_nbrs", C.c_int32), ("viscous_heating", C.c_int32),
                ("wall_visc", C.c_int32), ("n_materials", C.c_int32), ("reserved2", C.c_int32),
                ("mat_k", C.c_double * 8), ("mat_cp", C.c_double * 8)]


class Body(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("axis", C.c_double * 3), ("omega", C.c_double),
                ("T", C.c_double), ("k", C.c_double)]


class Report(C.Structure):
    _fields_ = [("t", C.c_double), ("step", C.c_int64), ("n_ac", C.c_int32), ("flags", C.c_int32),
                ("dt_ad", C.c_double), ("dt", C.c_double), ("vmax", C.c_double), ("mass", C.c_double),
                ("kinetic", C.c_double), ("thermal", C.c_double), ("heat_step", C.c_double),
                ("heat_total", C.c_double), ("mass_proxy", C.c_double), ("substeps", C.c_int64),
                ("diss_step", C.c_double), ("diss_total", C.c_double)]


class BodyReport(C.Structure):
    _fields_ = [("force", C.c_double * 3), ("torque", C.c_double * 3), ("torque_axis", C.c_double),
                ("power", C.c_double), ("heat_rate", C.c_double), ("torque_axis_int", C.c_double),
                ("energy_int", C.c_double), ("heat_int", C.c_double)]


SHAPES = {"sphere": 1, "box": 2, "cylinder": 3, "gear": 4}


class Shape(C.Structure):
    _fields_ = [("kind", C.c_int32), ("teeth", C.c_int32), ("inside", C.c_int32), ("reserved", C.c_int32),
                ("center", C.c_double * 3), ("size", C.c_double * 3), ("phase", C.c_double)]


class RelaxReport(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("bounded_last", C.c_int32), ("amax_first", C.c_double),
                ("amax_last", C.c_double), ("dt_last", C.c_double)]


def shape_struct(d: dict) -> Shape:
    """d: kind (sphere/box/cylinder/gear), center, size, teeth, phase, inside."""
    s = Shape()
    s.kind = SHAPES[d["kind"]]
    s.teeth = int(d.get("teeth", 0))
    s.inside = int(d.get("inside", 1))
    s.center[:] = [float(v) for v in d["center"]]
    s.size[:] = [float(v) for v in list(d["size"]) + [0.0] * (3 - len(d["size"]))]
    s.phase = float(d.get("phase", 0.0))
    return s


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


_lib = None


def lib():
    """Load libsph.so; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing")
        L = C.CDLL(LIB_PATH)
        L.sph_error_string.restype = C.c_char_p
        L.sph_last_error.restype = C.c_char_p
        L.sph_bytes_required.restype = C.c_size_t
        L.sph_bytes_required.argtypes = [C.POINTER(Params), C.c_int64, C.c_int64]
        _lib = L
    return _lib


EXPORTS = ["sph_error_string", "sph_last_error", "sph_create", "sph_set_bodies", "sph_set_fluid", "sph_set_solid",
           "sph_init", "sph_step", "sph_reduce", "sph_contact_factor", "sph_contact_factor_noalloc", "sph_relax", "sph_get_fluid", "sph_set_graph", "sph_set_timing",
           "sph_get_timing", "sph_dump_size", "sph_debug_dump", "sph_debug_poke_velocity", "sph_debug_set_fusion", "sph_destroy",
           "sph_bytes_required", "sph_pool_create", "sph_pool_admit", "sph_pool_step", "sph_pool_hold", "sph_pool_poll",
           "sph_pool_get_fluid", "sph_pool_release", "sph_pool_usage", "sph_pool_set_graph", "sph_pool_destroy"]


def check(rc, what=""):
    if rc != SPH_OK:
        L = lib()
        raise SphError(rc, f"{what}: {L.sph_error_string(rc).decode()}: {L.sph_last_error().decode()}")


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# ---------------------------------------------------------------------------
# device memory and streams from PyTorch
# ---------------------------------------------------------------------------
class TorchAllocator:
    """Routes the library's device allocations to torch's caching allocator."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = device

        def _alloc(nbytes, stream, user):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream))
            except Exception:  # reported to the caller as SPH_ERR_OOM
                return None

        def _free(ptr, stream, user):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:  # interpreter shutdown: torch already torn down
                pass

        self._a = ALLOC_FN(_alloc)
        self._f = FREE_FN(_free)
        self.struct = Allocator(self._a, self._f, None)


def params_struct(params: dict, precision="mixed", fixed_dt_ad=None, fixed_nac=None, **over) -> Params:
    d = dict(params)
    d.update(over)
    P = Params()
    for k in ("dp", "h_over_dp", "rho0", "c0", "nu", "k_f", "cp_f", "cfl_ad", "cfl_ac"):
        setattr(P, k, float(d[k]))
    for k in ("gravity", "grid_lo", "grid_hi"):
        getattr(P, k)[:] = [float(v) for v in d[k]]
    P.fixed_dt_ad = float(fixed_dt_ad if fixed_dt_ad is not None else d.get("fixed_dt_ad", 0.0))
    P.fixed_nac = int(fixed_nac if fixed_nac is not None else d.get("fixed_nac", 0))
    P.nac_max = int(d.get("nac_max", 16))
    P.free_surface = int(d.get("free_surface", 1))
    P.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    P.max_fluid_nbrs = int(d.get("max_fluid_nbrs", 0))
    P.max_solid_nbrs = int(d.get("max_solid_nbrs", 0))
    P.viscous_heating = int(d.get("viscous_heating", 0))
    P.wall_visc = int(d.get("wall_visc", 0))
    mats = d.get("materials") or []
    P.n_materials = len(mats)
    for m, (k, cp) in enumerate(mats):
        P.mat_k[m] = float(k)
        P.mat_cp[m] = float(cp)
    return P


def _material(case):
    m = getattr(case, "material", None)
    return None if m is None else np.ascontiguousarray(m, dtype=np.int32)


def bodies_array(bodies):
    arr = (Body * max(1, len(bodies)))()
    for i, b in enumerate(bodies):
        d = b.as_dict() if hasattr(b, "as_dict") else b
        arr[i].center[:] = list(d["center"])
        arr[i].axis[:] = list(d["axis"])
        arr[i].omega = d["omega"]
        arr[i].T = d["T"]
        arr[i].k = d["k"]
    return arr


def _report_dict(r: Report):
    return {k: getattr(r, k) for k, _ in Report._fields_}


def _body_dicts(br, n):
    out = []
    for b in range(n):
        x = br[b]
        out.append(dict(force=np.array(x.force[:]), torque=np.array(x.torque[:]), torque_axis=x.torque_axis,
                        power=x.power, heat_rate=x.heat_rate, torque_axis_int=x.torque_axis_int,
                        energy_int=x.energy_int, heat_int=x.heat_int))
    return out


class Solver:
    """One solve on the GPU: sph_create / set / init / step / reduce."""

    def __init__(self, case, precision="mixed", fixed_dt_ad=None, fixed_nac=None, stream=None, graph=True,
                 **param_over):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library needs an MI355X")
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.alloc = TorchAllocator(torch.cuda.current_device())
        self.nbody = len(case.bodies)
        self.nf = case.nf
        self.ns = case.ns
        self.P = params_struct(case.params, precision, fixed_dt_ad, fixed_nac, **param_over)
        L = lib()
        h = C.c_void_p()
        check(L.sph_create(C.byref(self.P), C.byref(self.alloc.struct), C.c_void_p(self.stream.cuda_stream),
                           C.byref(h)), "sph_create")
        self.h = h
        B = bodies_array(case.bodies)
        check(L.sph_set_bodies(h, C.c_int32(self.nbody), B), "sph_set_bodies")
        x, v, r, T = _f64(case.xf, (-1, 3)), _f64(case.vf, (-1, 3)), _f64(case.rhof), _f64(case.Tf)
        mat = _material(case)
        check(L.sph_set_fluid(h, C.c_int64(self.nf), _p(x), _p(v), _p(r), _p(T), _p(mat) if mat is not None else None),
              "sph_set_fluid")
        x0, n0 = _f64(case.xs0, (-1, 3)), _f64(case.ns0, (-1, 3))
        body = np.ascontiguousarray(case.body, dtype=np.int32)
        check(L.sph_set_solid(h, C.c_int64(self.ns), _p(x0), _p(n0), _p(body)), "sph_set_solid")
        if not graph:
            check(L.sph_set_graph(h, C.c_int32(0)), "sph_set_graph")
        check(L.sph_init(h), "sph_init")

    def step(self, n=1):
        check(lib().sph_step(self.h, C.c_int32(n)), "sph_step")

    def reduce(self, raise_on_fault=True):
        r = Report()
        br = (BodyReport * max(1, self.nbody))()
        rc = lib().sph_reduce(self.h, C.byref(r), br)
        out = _report_dict(r)
        out["bodies"] = _body_dicts(br, self.nbody)
        out["rc"] = rc
        if raise_on_fault:
            check(rc, "sph_reduce")
        return out

    def get_fluid(self):
        x = np.zeros((self.nf, 3))
        v = np.zeros((self.nf, 3))
        r = np.zeros(self.nf)
        T = np.zeros(self.nf)
        check(lib().sph_get_fluid(self.h, _p(x), _p(v), _p(r), _p(T)), "sph_get_fluid")
        return dict(x=x, v=v, rho=r, T=T)

    def contact_factor(self):
        """Contact factor of every solid particle at the current time (eq. 24),
        in the case's solid order, and its mean per body."""
        z = np.zeros(max(self.ns, 1))
        m = np.zeros(max(self.nbody, 1))
        check(lib().sph_contact_factor(self.h, _p(z), _p(m)), "sph_contact_factor")
        return z[: self.ns], m[: self.nbody]

    def contact_factor_noalloc(self, zeta=None, body_mean=None):
        """The allocation-free contact factor: writes into caller-owned torch
        float64 device tensors (ns and nbody elements, either may be None)
        on the solver's stream, asynchronously; the caller synchronises."""
        import torch
        for t, n in ((zeta, self.ns), (body_mean, self.nbody)):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()
                                  or t.numel() < n):
                raise ValueError("outputs must be contiguous float64 device tensors of the right size")
        check(lib().sph_contact_factor_noalloc(self.h, C.c_void_p(zeta.data_ptr() if zeta is not None else 0),
                                               C.c_void_p(body_mean.data_ptr() if body_mean is not None else 0)),
              "sph_contact_factor_noalloc")

    def relax(self, shape: dict, iterations: int):
        """Physics-driven relaxation (Section 2.2) of the fluid particles inside
        `shape`; positions change in place (read them with get_fluid)."""
        r = RelaxReport()
        check(lib().sph_relax(self.h, C.byref(shape_struct(shape)), C.c_int32(int(iterations)), C.byref(r)),
              "sph_relax")
        return {k: getattr(r, k) for k, _ in RelaxReport._fields_}

    def set_fusion(self, on=True):
        """Run the first sub-step inside the viscous/heat sweep (default) or unfused."""
        check(lib().sph_debug_set_fusion(self.h, C.c_int32(1 if on else 0)), "sph_debug_set_fusion")

    def set_timing(self, on=True):
        check(lib().sph_set_timing(self.h, C.c_int32(int(on))), "sph_set_timing")

    def timing(self, kernel):
        kid = K[kernel] if isinstance(kernel, str) else int(kernel)
        n = C.c_int32()
        check(lib().sph_get_timing(self.h, C.c_int32(kid), C.c_int32(0), None, C.byref(n)), "sph_get_timing")
        buf = np.zeros(max(1, n.value), dtype=np.float32)
        check(lib().sph_get_timing(self.h, C.c_int32(kid), C.c_int32(n.value), _p(buf), C.byref(n)),
              "sph_get_timing")
        return buf[: n.value].astype(np.float64)

    def dump(self, what):
        code = DUMP[what]
        nb = C.c_size_t()
        check(lib().sph_dump_size(self.h, C.c_int32(code), C.byref(nb)), "sph_dump_size")
        raw = np.zeros(nb.value, dtype=np.uint8)
        check(lib().sph_debug_dump(self.h, C.c_int32(code), _p(raw), nb), "sph_debug_dump")
        if what in ("fluid_ids", "solid_ids", "fluid_cell", "nbr_count", "nbr_fluid", "nbr_solid"):
            return raw.view(np.uint32)
        return raw.view(np.float64)

    def poke_velocity(self, original_index, v3):
        v = _f64(v3)
        check(lib().sph_debug_poke_velocity(self.h, C.c_int64(original_index), _p(v)), "sph_debug_poke_velocity")

    # --- neighbour rows in original-index terms, for parity tests -------------
    def neighbour_sets(self):
        fid = self.dump("fluid_ids").astype(np.int64)
        sid = self.dump("solid_ids").astype(np.int64)
        cnt = self.dump("nbr_count").reshape(2, self.nf)
        kf = len(self.dump("nbr_fluid")) // self.nf
        ks = len(self.dump("nbr_solid")) // self.nf
        rf = self.dump("nbr_fluid").reshape(self.nf, kf)
        rs = self.dump("nbr_solid").reshape(self.nf, ks)
        fl = [None] * self.nf
        so = [None] * self.nf
        for k in range(self.nf):
            o = fid[k]
            fl[o] = frozenset(fid[rf[k, : cnt[0, k]]].tolist())
            so[o] = frozenset(sid[rs[k, : cnt[1, k]]].tolist())
        return fl, so

    def close(self):
        if getattr(self, "h", None):
            lib().sph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """Many solves stepped together in batched launches (sph_pool_*)."""

    def __init__(self, hbm_budget, max_slots=16, precision="mixed", stream=None, graph=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library needs an MI355X")
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.alloc = TorchAllocator(torch.cuda.current_device())
        self.precision = PREC[precision] if isinstance(precision, str) else int(precision)
        h = C.c_void_p()
        check(lib().sph_pool_create(C.c_size_t(int(hbm_budget)), C.c_int32(max_slots), C.c_int32(self.precision),
                                    C.byref(self.alloc.struct), C.c_void_p(self.stream.cuda_stream), C.byref(h)),
              "sph_pool_create")
        self.h = h
        self.nbody = {}
        self.nf = {}
        if not graph:
            check(lib().sph_pool_set_graph(h, C.c_int32(0)), "sph_pool_set_graph")

    @staticmethod
    def bytes_required(case, precision="mixed"):
        P = params_struct(case.params, precision)
        return int(lib().sph_bytes_required(C.byref(P), C.c_int64(case.nf), C.c_int64(case.ns)))

    def admit(self, case, target_steps, **param_over):
        """Returns the slot index, or None when the pool has no room now."""
        P = params_struct(case.params, self.precision, **param_over)
        B = bodies_array(case.bodies)
        x, v, r, T = _f64(case.xf, (-1, 3)), _f64(case.vf, (-1, 3)), _f64(case.rhof), _f64(case.Tf)
        x0, n0 = _f64(case.xs0, (-1, 3)), _f64(case.ns0, (-1, 3))
        body = np.ascontiguousarray(case.body, dtype=np.int32)
        slot = C.c_int32(-1)
        mat = _material(case)
        rc = lib().sph_pool_admit(self.h, C.byref(P), C.c_int32(len(case.bodies)), B, C.c_int64(case.nf), _p(x),
                                  _p(v), _p(r), _p(T), _p(mat) if mat is not None else None, C.c_int64(case.ns),
                                  _p(x0), _p(n0), _p(body), C.c_int64(int(target_steps)), C.byref(slot))
        if rc == SPH_ERR_BUDGET:
            return None
        check(rc, "sph_pool_admit")
        self.nbody[slot.value] = len(case.bodies)
        self.nf[slot.value] = case.nf
        return slot.value

    def step(self, n=1):
        check(lib().sph_pool_step(self.h, C.c_int32(n)), "sph_pool_step")

    def hold(self, slot, hold=True):
        """Leave the slot out of later steps (hold=True) or step it again (False)."""
        check(lib().sph_pool_hold(self.h, C.c_int32(slot), C.c_int32(1 if hold else 0)), "sph_pool_hold")

    def poll(self, slot):
        """(done, report or None); a faulted slot reports done with report['rc'] != 0."""
        done = C.c_int32(0)
        r = Report()
        nb = self.nbody[slot]
        br = (BodyReport * max(1, nb))()
        rc = lib().sph_pool_poll(self.h, C.c_int32(slot), C.byref(done), C.byref(r), br)
        if rc not in (SPH_OK, SPH_ERR_DOMAIN, SPH_ERR_NONFINITE, SPH_ERR_CAPACITY):
            check(rc, "sph_pool_poll")
        if not done.value:
            return False, None
        out = _report_dict(r)
        out["bodies"] = _body_dicts(br, nb)
        out["rc"] = rc
        return True, out

    def get_fluid(self, slot):
        n = self.nf[slot]
        x = np.zeros((n, 3))
        v = np.zeros((n, 3))
        r = np.zeros(n)
        T = np.zeros(n)
        check(lib().sph_pool_get_fluid(self.h, C.c_int32(slot), _p(x), _p(v), _p(r), _p(T)), "sph_pool_get_fluid")
        return dict(x=x, v=v, rho=r, T=T)

    def release(self, slot):
        check(lib().sph_pool_release(self.h, C.c_int32(slot)), "sph_pool_release")
        self.nbody.pop(slot, None)
        self.nf.pop(slot, None)

    def usage(self):
        b = C.c_size_t()
        a = C.c_int32()
        check(lib().sph_pool_usage(self.h, C.byref(b), C.byref(a)), "sph_pool_usage")
        return b.value, a.value

    def close(self):
        if getattr(self, "h", None):
            lib().sph_pool_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
