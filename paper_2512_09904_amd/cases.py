"""Seeded synthetic case generators for the gearbox SPH hot path.

This module only builds initial particle sets: lattices, wall layers, rotating
solid shells with outward normals, hydrostatic initial density and the
parameter sets of the workloads.  It contains none of the solver's per-step
arithmetic (kernel, Riemann solver, sweeps, integrator), so both the FP64 CPU
oracle and the HIP library can be driven from the same inputs without sharing
any code of the method.

Geometry and property choices follow the paper's problem statement:
material properties (Table 6), operating ranges (Table 5: speeds 150-1500
rad/s, lubrication depth, viscosity 15-44 mm^2/s), particle spacings
(Section 4.3: dp 0.8-2 mm), smoothing length h = 1.3 dp, c0 = 10 Umax (eq. 2)
and the two-slab conduction benchmark (Section 3.2, Table 3).  The paper's
CAD gearbox is not available; toothed disks stand in for the gears.

Random jitter comes from SplitMix64 (Steele, Lea, Flood 2014) keyed on
(seed, particle id, axis), so a case is reproducible bit for bit.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

GRAVITY = (0.0, 0.0, -9.81)      # z up; magnitude not stated by the paper
KELVIN = 273.15

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied elementwise to uint64 inputs."""
    z = (x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15))
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def uniform01(seed: int, ids: np.ndarray, axis: int) -> np.ndarray:
    """U[0,1) doubles from SplitMix64(SplitMix64(seed) xor (3 id + axis))."""
    with np.errstate(over="ignore"):
        s = splitmix64(np.array([seed], dtype=np.uint64))[0]
        key = ids.astype(np.uint64) * np.uint64(3) + np.uint64(axis)
        u = splitmix64(key ^ s)
    return (u >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def jitter(seed: int, n: int, dp: float, amp: float = 0.05) -> np.ndarray:
    """Per-particle offsets U(-amp, amp) * dp on each axis."""
    ids = np.arange(n, dtype=np.uint64)
    out = np.empty((n, 3))
    for a in range(3):
        out[:, a] = (uniform01(seed, ids, a) - 0.5) * (2.0 * amp * dp)
    return out


@dataclasses.dataclass
class Body:
    center: tuple
    axis: tuple
    omega: float
    T: float
    k: float

    def as_dict(self):
        return dict(center=tuple(map(float, self.center)), axis=tuple(map(float, self.axis)),
                    omega=float(self.omega), T=float(self.T), k=float(self.k))


@dataclasses.dataclass
class Case:
    """A complete initial condition: parameters, bodies, fluid and solid particles.

    Fluid arrays: xf (nf,3), vf (nf,3), rhof (nf,), Tf (nf,).
    Solid arrays: xs0 (ns,3) positions at t = 0, ns0 (ns,3) unit normals
    pointing into the fluid, body (ns,) int32 index into ``bodies``.
    Body 0 is the static housing.
    """
    name: str
    params: dict
    bodies: List[Body]
    xf: np.ndarray
    vf: np.ndarray
    rhof: np.ndarray
    Tf: np.ndarray
    xs0: np.ndarray
    ns0: np.ndarray
    body: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)
    material: Optional[np.ndarray] = None   # fluid material index per particle (params["materials"])

    @property
    def nf(self) -> int:
        return int(self.xf.shape[0])

    @property
    def ns(self) -> int:
        return int(self.xs0.shape[0])

    def copy(self) -> "Case":
        return dataclasses.replace(
            self, params=dict(self.params), bodies=[dataclasses.replace(b) for b in self.bodies],
            xf=self.xf.copy(), vf=self.vf.copy(), rhof=self.rhof.copy(), Tf=self.Tf.copy(),
            xs0=self.xs0.copy(), ns0=self.ns0.copy(), body=self.body.copy(), meta=dict(self.meta),
            material=None if self.material is None else self.material.copy())


def default_params(dp: float, rho0: float, c0: float, nu: float, k_f: float, cp_f: float,
                   lo, hi, h_over_dp: float = 1.3, free_surface: int = 1,
                   gravity=GRAVITY) -> dict:
    """Solver parameters; the grid spans the walls plus one spare cell of size 2h."""
    cs = 2.0 * h_over_dp * dp
    glo = tuple(float(l - cs) for l in lo)
    ghi = tuple(float(u + cs) for u in hi)
    return dict(dp=float(dp), h_over_dp=float(h_over_dp), rho0=float(rho0), c0=float(c0),
                nu=float(nu), k_f=float(k_f), cp_f=float(cp_f), gravity=tuple(gravity),
                grid_lo=glo, grid_hi=ghi, free_surface=int(free_surface),
                cfl_ad=0.25, cfl_ac=0.6, nac_max=16, fixed_dt_ad=0.0, fixed_nac=0)


# ----------------------------------------------------------------------------
# lattice helpers
# ----------------------------------------------------------------------------

def _box_lattice(n, dp, pad):
    """Integer lattice indices i in [-pad, n+pad) per axis, site at (i + 1/2) dp."""
    rng = [np.arange(-pad, n[a] + pad) for a in range(3)]
    I, J, K = np.meshgrid(*rng, indexing="ij")
    idx = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    return idx, (idx + 0.5) * dp


def _walls(n, dp, layers=3):
    """Closed box of `layers` lattice layers outside [0, n dp); inward normals."""
    idx, x = _box_lattice(n, dp, layers)
    nrm = np.zeros_like(x)
    outside = np.zeros(len(idx), dtype=bool)
    for a in range(3):
        lo = idx[:, a] < 0
        hi = idx[:, a] >= n[a]
        nrm[lo, a] += 1.0
        nrm[hi, a] -= 1.0
        outside |= lo | hi
    x, nrm = x[outside], nrm[outside]
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    return x, nrm


def _ball_offsets(radius):
    r = int(math.ceil(radius))
    g = np.arange(-r, r + 1)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    off = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    d = np.linalg.norm(off, axis=1)
    keep = (d <= radius) & (d > 0)
    return off[keep], d[keep]


def _shell_and_normals(inside_fn, lo_idx, hi_idx, dp, layers=3):
    """Lattice sites inside a body and within `layers` spacings of its surface.

    `inside_fn(x)` -> bool array.  Normals point out of the body (into the
    fluid): the direction of the weighted sum of offsets to outside sites
    within radius layers + 1.
    """
    from scipy import ndimage
    pad = layers + 2
    rng = [np.arange(lo_idx[a] - pad, hi_idx[a] + pad) for a in range(3)]
    shape = tuple(len(r) for r in rng)
    I, J, K = np.meshgrid(*rng, indexing="ij")
    x = (np.stack([I, J, K], axis=-1) + 0.5) * dp
    inside = inside_fn(x.reshape(-1, 3)).reshape(shape)
    outside = ~inside
    off, d = _ball_offsets(layers)
    ball = np.zeros((2 * layers + 1,) * 3, dtype=bool)
    ball[tuple((off + layers).T)] = True
    near_out = ndimage.binary_dilation(outside, structure=ball)
    shell = inside & near_out
    R = layers + 1
    offn, dn = _ball_offsets(R)
    w = (1.0 - dn / (R + 1.0)) ** 2
    grad = np.zeros(shape + (3,))
    o = outside.astype(np.float64)
    for a in range(3):
        kern = np.zeros((2 * R + 1,) * 3)
        kern[tuple((offn + R).T)] = offn[:, a] * w
        grad[..., a] = ndimage.correlate(o, kern, mode="constant", cval=1.0)
    xs = x[shell]
    ns = grad[shell]
    nn = np.linalg.norm(ns, axis=1)
    ns = ns / np.where(nn > 0, nn, 1.0)[:, None]
    return xs, ns


def disk_inside(center, radius, thickness):
    c = np.asarray(center, dtype=np.float64)

    def f(x):
        d = x - c
        return ((d[:, 0] ** 2 + d[:, 2] ** 2) <= radius * radius) & (np.abs(d[:, 1]) <= 0.5 * thickness)
    return f


def gear_inside(center, z_teeth, r_tip, r_root, face, phase, tooth_frac=0.5):
    """Spur-gear proxy about an axis parallel to y: tooth where
    frac(z th/2pi + tooth_frac/2 + phase) < tooth_frac (teeth of tooth_frac of
    the pitch, centred on th = 0 at phase 0; 1/2 gives the survey's teeth)."""
    c = np.asarray(center, dtype=np.float64)

    def f(x):
        d = x - c
        r2 = d[:, 0] ** 2 + d[:, 2] ** 2
        th = np.arctan2(d[:, 2], d[:, 0])
        fr = np.mod(z_teeth * th / (2.0 * math.pi) + 0.5 * tooth_frac + phase, 1.0)
        tooth = fr < tooth_frac
        inr = (r2 <= r_root * r_root) | ((r2 <= r_tip * r_tip) & tooth)
        return inr & (np.abs(d[:, 1]) <= 0.5 * face)
    return f


def _idx_bounds(center, half_extent, dp):
    c = np.asarray(center)
    e = np.asarray(half_extent)
    lo = np.floor((c - e) / dp).astype(int) - 1
    hi = np.ceil((c + e) / dp).astype(int) + 1
    return lo, hi


# ----------------------------------------------------------------------------
# tank with rotating bodies
# ----------------------------------------------------------------------------

def _tank(name, box, dp, fill_h, bodies_geo, rho0, nu, k_f, cp_f, T_oil, T_wall, k_solid,
          seed, umax=None, c0=None, jitter_amp=0.05, h_over_dp=1.3, free_surface=1,
          gravity=GRAVITY):
    n = tuple(int(round(b / dp)) for b in box)
    L = tuple(n[a] * dp for a in range(3))
    # fluid: box interior below the free surface, outside every body
    idx, x = _box_lattice(n, dp, 0)
    keep = x[:, 2] < fill_h
    for geo in bodies_geo:
        keep &= ~geo["inside"](x)
    xf = x[keep]
    xw, nw = _walls(n, dp)
    bodies = [Body(center=(0.0, 0.0, 0.0), axis=(0.0, 0.0, 1.0), omega=0.0, T=T_wall, k=k_solid)]
    xs_list, ns_list, b_list = [xw], [nw], [np.zeros(len(xw), dtype=np.int32)]
    tip = 0.0
    for bi, geo in enumerate(bodies_geo, start=1):
        lo, hi = _idx_bounds(geo["center"], geo["half_extent"], dp)
        xs, ns = _shell_and_normals(geo["inside"], lo, hi, dp)
        xs_list.append(xs)
        ns_list.append(ns)
        b_list.append(np.full(len(xs), bi, dtype=np.int32))
        bodies.append(Body(center=tuple(geo["center"]), axis=(0.0, 1.0, 0.0), omega=geo["omega"],
                           T=geo.get("T", T_wall), k=k_solid))
        tip = max(tip, abs(geo["omega"]) * geo["r_tip"])
    if umax is None:
        umax = tip if tip > 0 else math.sqrt(2.0 * abs(gravity[2]) * fill_h)
    if c0 is None:
        c0 = 10.0 * umax
    xf = xf + jitter(seed, len(xf), dp, jitter_amp)
    g = abs(gravity[2])
    rhof = rho0 + rho0 * g * np.maximum(fill_h - xf[:, 2], 0.0) / (c0 * c0)
    params = default_params(dp, rho0, c0, nu, k_f, cp_f, (0.0, 0.0, 0.0), L,
                            h_over_dp=h_over_dp, free_surface=free_surface, gravity=gravity)
    params["grid_lo"] = tuple(v - 3 * dp for v in params["grid_lo"])
    params["grid_hi"] = tuple(v + 3 * dp for v in params["grid_hi"])
    case = Case(name=name, params=params, bodies=bodies, xf=np.ascontiguousarray(xf),
                vf=np.zeros_like(xf), rhof=rhof, Tf=np.full(len(xf), float(T_oil)),
                xs0=np.ascontiguousarray(np.concatenate(xs_list)),
                ns0=np.ascontiguousarray(np.concatenate(ns_list)),
                body=np.concatenate(b_list).astype(np.int32),
                meta=dict(box=L, fill_h=fill_h, umax=umax, seed=seed))
    return case


def tank_c1(seed: int = 0, dp: float = 2e-3, omega: float = 150.0) -> Case:
    """Plain WCSPH tank: 0.10 x 0.05 x 0.05 m, 40 % oil fill, one disk r = 15 mm."""
    geo = dict(center=(0.05, 0.025, 0.025), half_extent=(0.015, 0.005, 0.015), r_tip=0.015,
               omega=omega, inside=disk_inside((0.05, 0.025, 0.025), 0.015, 0.010))
    return _tank("tank_c1", (0.10, 0.05, 0.05), dp, 0.02, [geo], rho0=870.0, nu=1e-4,
                 k_f=0.13, cp_f=2000.0, T_oil=40.0 + KELVIN, T_wall=60.0 + KELVIN,
                 k_solid=20.0, seed=seed)


def still_tank(seed: int = 0, dp: float = 2e-3, box=(0.10, 0.05, 0.05), fill=0.02,
               c0: float = 22.5, jitter_amp: float = 0.05) -> Case:
    """Hydrostatic tank without bodies, c0 of the C1 tank kept."""
    return _tank("still_tank", box, dp, fill, [], rho0=870.0, nu=1e-4, k_f=0.13, cp_f=2000.0,
                 T_oil=40.0 + KELVIN, T_wall=40.0 + KELVIN, k_solid=20.0, seed=seed,
                 umax=c0 / 10.0, c0=c0, jitter_amp=jitter_amp)


def gearbox(seed: int = 0, dp: float = 1.5e-3, omega_big: float = 300.0, immersion: float = 0.030,
            nu: float = 1e-4, box=(0.30, 0.15, 0.20), tooth_frac: float = 0.5,
            centre_distance: float = 0.120) -> Case:
    """Gearbox proxy: two meshing toothed disks (20/40 teeth, module 4 mm), axes parallel to y.

    The 40-tooth gear turns at omega_big, the 20-tooth gear at -2 omega_big; the
    free surface sits `immersion` below the gear centres (paper's lubrication
    depth convention).  Teeth span tooth_frac of the pitch, rectangular in
    angle; the gears sit centre_distance apart (their pitch circles touch at
    0.120 m).
    """
    m = 4e-3
    zc = 0.100
    yc = box[1] / 2.0
    face = 0.030
    g1 = dict(center=(0.070, yc, zc), z=20, phase=0.0, omega=-2.0 * omega_big)
    g2 = dict(center=(0.070 + centre_distance, yc, zc), z=40, phase=0.5, omega=omega_big)
    geos = []
    for g in (g1, g2):
        rp = m * g["z"] / 2.0
        ra, rf = rp + m, rp - 1.25 * m
        geos.append(dict(center=g["center"], half_extent=(ra, face / 2, ra), r_tip=ra, omega=g["omega"],
                         inside=gear_inside(g["center"], g["z"], ra, rf, face, g["phase"], tooth_frac)))
    return _tank("gearbox", box, dp, zc - immersion, geos, rho0=870.0, nu=nu, k_f=0.13, cp_f=2000.0,
                 T_oil=40.0 + KELVIN, T_wall=60.0 + KELVIN, k_solid=20.0, seed=seed)


def gearbox_c2(seed: int = 0) -> Case:
    """1.5 mm gearbox proxy at 300 rad/s, 30 mm immersion, nu = 1e-4 (about 1.4 M particles)."""
    c = gearbox(seed=seed, dp=1.5e-3, omega_big=300.0, immersion=0.030, nu=1e-4)
    c.name = "gearbox_c2"
    return c


def gearbox_c3(seed: int = 0, dp: float = 1e-3) -> Case:
    """Full-size proxy: 1 mm spacing, 600 rad/s, nu = 2.2e-4, 50 mm immersion."""
    c = gearbox(seed=seed, dp=dp, omega_big=600.0, immersion=0.050, nu=2.2e-4)
    c.name = "gearbox_c3"
    return c


def serving_tank(n_fluid: int, omega: float, immersion: float, nu: float, seed: int = 0) -> Case:
    """Serving request: 0.20 x 0.10 x 0.15 m tank, disk r = 40 mm, thickness 20 mm at z = 0.075.

    The free surface sits `immersion` above the disk's lowest point; dp is chosen
    so that the fluid holds about `n_fluid` particles.
    """
    box = (0.20, 0.10, 0.15)
    H = 0.035 + immersion
    vol = box[0] * box[1] * H
    dp = (vol / float(n_fluid)) ** (1.0 / 3.0)
    geo = dict(center=(0.10, 0.05, 0.075), half_extent=(0.04, 0.01, 0.04), r_tip=0.04, omega=omega,
               inside=disk_inside((0.10, 0.05, 0.075), 0.040, 0.020))
    c = _tank("serving_tank", box, dp, H, [geo], rho0=870.0, nu=nu, k_f=0.13, cp_f=2000.0,
              T_oil=40.0 + KELVIN, T_wall=60.0 + KELVIN, k_solid=20.0, seed=seed)
    c.meta.update(omega=omega, immersion=immersion, nu=nu, n_request=n_fluid)
    return c


def sphere_couette(dp: float = 0.625e-3, R1: float = 5e-3, R2: float = 10e-3, omega: float = 1.0,
                   nu: float = 1e-2, rho0: float = 870.0, c0: float = 1.0) -> Case:
    """Fluid between an inner sphere spinning about z and a fixed outer sphere, no gravity."""
    c = np.array([0.0, 0.0, 0.0])
    n = int(math.ceil((R2 + 4 * dp) / dp))
    g = np.arange(-n, n)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    x = (np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1) + 0.5) * dp
    r = np.linalg.norm(x - c, axis=1)
    fluid = (r > R1) & (r < R2)
    inner = (r <= R1) & (r > R1 - 3 * dp)
    outer = (r >= R2) & (r < R2 + 3 * dp)
    xf = x[fluid]
    xs = np.concatenate([x[outer], x[inner]])
    nrm = np.concatenate([-(x[outer] - c) / r[outer][:, None], (x[inner] - c) / r[inner][:, None]])
    body = np.concatenate([np.zeros(outer.sum(), np.int32), np.ones(inner.sum(), np.int32)])
    lo = (-(R2 + 3 * dp),) * 3
    hi = ((R2 + 3 * dp),) * 3
    params = default_params(dp, rho0, c0, nu, 0.13, 2000.0, lo, hi, free_surface=0,
                            gravity=(0.0, 0.0, 0.0))
    bodies = [Body((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), 0.0, 313.15, 20.0),
              Body((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), omega, 313.15, 20.0)]
    return Case("sphere_couette", params, bodies, np.ascontiguousarray(xf), np.zeros_like(xf),
                np.full(len(xf), rho0), np.full(len(xf), 313.15), np.ascontiguousarray(xs),
                np.ascontiguousarray(nrm), body, meta=dict(R1=R1, R2=R2, omega=omega))


def slab(nx: int = 80, ny: int = 40, nz: int = 8, dx: float = 0.0125):
    """Two-slab conduction benchmark (Section 3.2, Table 3): interface at x = 0.5.

    Returns positions and per-particle material properties (rho, k, cp, T0).
    Left material: rho 1000, k 1, cp 1, T 0; right: rho 2000, k 3, cp 1, T 1.
    """
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    x = (np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1) + 0.5) * dx
    right = x[:, 0] > 0.5
    rho = np.where(right, 2000.0, 1000.0)
    k = np.where(right, 3.0, 1.0)
    cp = np.ones(len(x))
    T0 = np.where(right, 1.0, 0.0)
    return dict(x=np.ascontiguousarray(x), rho=rho, k=k, cp=cp, T=T0, dx=dx,
                lo=(-2 * dx, -2 * dx, -2 * dx), hi=(nx * dx + 2 * dx, ny * dx + 2 * dx, nz * dx + 2 * dx))


def lattice_block(n: int, dp: float = 1.0, jitter_amp: float = 0.0, seed: int = 0):
    """Cubic block of n^3 lattice sites at (i + 1/2) dp, optionally jittered."""
    g = np.arange(n)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    x = (np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1) + 0.5) * dp
    if jitter_amp > 0:
        x = x + jitter(seed, len(x), dp, jitter_amp)
    return np.ascontiguousarray(x)


def random_box(n: int, L: float, seed: int = 0) -> np.ndarray:
    """n uniform random points in [0, L)^3 from SplitMix64."""
    ids = np.arange(n, dtype=np.uint64)
    return np.ascontiguousarray(np.stack([uniform01(seed, ids, a) * L for a in range(3)], axis=1))


def sub_box(case: Case, center, half, halo: float) -> dict:
    """Indices of fluid particles inside a box and of those in a read-only halo around it."""
    c = np.asarray(center)
    h = np.asarray(half)
    d = np.abs(case.xf - c)
    core = np.all(d <= h, axis=1)
    halo_m = np.all(d <= h + halo, axis=1) & ~core
    return dict(core=np.nonzero(core)[0], halo=np.nonzero(halo_m)[0])


# ----------------------------------------------------------------------------
# particle relaxation (Section 2.2): lattice sites inside an analytic shape
# ----------------------------------------------------------------------------

def shape_inside(shape: dict):
    """Inside test of an analytic shape (the dict of the relaxation calls):
    sphere, box, cylinder or gear, axis along y for the last two."""
    c = np.asarray(shape["center"], dtype=np.float64)
    s = list(shape["size"]) + [0.0] * (3 - len(shape["size"]))
    k = shape["kind"]
    if k == "sphere":
        f = lambda x: np.sum((x - c) ** 2, axis=1) < s[0] ** 2
    elif k == "box":
        f = lambda x: np.all(np.abs(x - c) < np.asarray(s[:3]), axis=1)
    elif k == "cylinder":
        f = lambda x: (((x[:, 0] - c[0]) ** 2 + (x[:, 2] - c[2]) ** 2) < s[0] ** 2) & (np.abs(x[:, 1] - c[1]) < s[1])
    elif k == "gear":
        f = gear_inside(c, int(shape["teeth"]), s[0], s[1], 2.0 * s[2], float(shape.get("phase", 0.0)))
    else:
        raise ValueError(k)
    if int(shape.get("inside", 1)):
        return f
    return lambda x: ~f(x)


def relax_case(shape: dict, dp: float, bound: float, jitter_amp: float = 0.25, seed: int = 0,
               h_over_dp: float = 1.3) -> Case:
    """Initial particles of a relaxation: the sites (i + 1/2) dp of the lattice
    inside `shape`, within the cube [-bound, bound]^3 around the shape's
    centre, moved by a seeded jitter of +-jitter_amp dp per axis (the start of
    eq. 6's relaxation: a lattice embedded in the geometry).  Carried as the
    fluid of a case with one static body and no solid particles."""
    c = np.asarray(shape["center"], dtype=np.float64)
    lo_i = np.floor((c - bound) / dp).astype(int)
    hi_i = np.ceil((c + bound) / dp).astype(int)
    rng = [np.arange(lo_i[a], hi_i[a]) for a in range(3)]
    I, J, K = np.meshgrid(*rng, indexing="ij")
    x = (np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1) + 0.5) * dp
    x = x[shape_inside(shape)(x)]
    if jitter_amp > 0:
        x = x + jitter(seed, len(x), dp, jitter_amp)
    n = len(x)
    params = default_params(dp, 1000.0, 10.0, 1e-4, 0.13, 2000.0, tuple(c - bound - dp), tuple(c + bound + dp),
                            h_over_dp=h_over_dp, gravity=(0.0, 0.0, 0.0))
    return Case(name=f"relax-{shape['kind']}", params=params,
                bodies=[Body(tuple(c), (0.0, 1.0, 0.0), 0.0, 300.0, 20.0)],
                xf=np.ascontiguousarray(x), vf=np.zeros((n, 3)), rhof=np.full(n, 1000.0), Tf=np.full(n, 300.0),
                xs0=np.zeros((0, 3)), ns0=np.zeros((0, 3)), body=np.zeros(0, np.int32),
                meta=dict(shape=dict(shape), umax=1.0))
