"""Multi-step pins of the FP64 oracle: hydrostatics, eq. 13 sign, rotating walls.

These run the full advection step of the oracle (Sections 2.3-2.8 of
arXiv 2512.09904) on small synthetic tanks.
"""
import math

import numpy as np
import pytest

from paper_2512_09904_amd import cases


def _hydro_error(s, c, H):
    rho0 = c.params["rho0"]
    g = abs(c.params["gravity"][2])
    c0 = c.params["c0"]
    dp = c.params["dp"]
    box = c.meta["box"]
    x = s.x
    p = c0 * c0 * (s.rho - rho0)
    away = np.ones(len(x), bool)
    for a in range(2):
        away &= (x[:, a] > 3 * dp) & (x[:, a] < box[a] - 3 * dp)
    away &= (x[:, 2] > 3 * dp) & (x[:, 2] < H - 2 * 1.3 * dp)
    e = (p - rho0 * g * (H - x[:, 2]))[away] / (rho0 * g * H)
    zb = np.floor(x[away, 2] / dp)
    return max(abs(e[zb == b].mean()) for b in np.unique(zb))


def test_still_tank_stays_hydrostatic(ora):
    """Walls (eq. 16-19), EoS (eq. 2), gravity and density re-initialisation
    (eq. 14), 2000 advection steps (32,000 acoustic sub-steps, 2.2 s) of a
    still tank:
    - |v|max stays below 1 % of the reference speed c0/10 once the jittered
      lattice has settled (P8), and the mass is exact;
    - at step 600 the pressure of every depth bin away from the walls is
      within 1 % of rho0 g (H - z) (P11);
    - after that the max of eq. 14 ratchets the density up (every upward
      fluctuation of the kernel sum is kept): the mean pressure rises at a
      slowly growing rate below 3 % of rho0 g H per simulated second
      (1.5-2.5 % measured; 7 % of rho0 g H at step 2000), and the mass proxy
      by less than 2e-5.  Applying eq. 14 only where the kernel sum is
      deficient and eq. 15 elsewhere stops the rise but leaves the depth bins
      5-6 % off, so the literal reading is kept."""
    H = 0.02
    c = cases.still_tank(dp=2e-3, box=(0.04, 0.02, 0.03), fill=H)
    s = ora.State(c)
    umax = c.params["c0"] / 10.0
    rho0, g, c0 = c.params["rho0"], abs(c.params["gravity"][2]), c.params["c0"]
    m0 = None
    mean_p = {}
    for k in range(2000):
        r = s.step()
        m0 = m0 or r["mass"]
        if k >= 50:          # after the jittered lattice has settled
            assert r["vmax"] <= 1e-2 * umax, (k, r["vmax"])
        assert r["mass"] == m0
        if k + 1 == 600:
            assert _hydro_error(s, c, H) <= 0.01
            proxy600 = r["mass_proxy"] / r["mass"] - 1.0
        if (k + 1) % 200 == 0:
            mean_p[k + 1] = (float(np.mean(c0 * c0 * (s.rho - rho0))) / (rho0 * g * H), r["t"])
    ks = sorted(k for k in mean_p if k >= 600)
    rates = [(mean_p[b][0] - mean_p[a][0]) / (mean_p[b][1] - mean_p[a][1]) for a, b in zip(ks, ks[1:])]
    assert all(0.0 < q < 0.03 for q in rates), rates
    assert abs((r["mass_proxy"] / r["mass"] - 1.0) - proxy600) < 2e-5


def test_printed_eq13_sign_is_unstable(ora):
    """The sign of eq. 13 as printed makes pressure anti-diffusive: the still tank blows up."""
    c = cases.still_tank(dp=2e-3, box=(0.04, 0.02, 0.03), fill=0.02)
    s = ora.State(c, eq13_printed=1)
    blew = False
    for _ in range(20):
        try:
            r = s.step()
        except RuntimeError:
            blew = True
            break
        if not np.isfinite(r["vmax"]) or r["vmax"] > 1.0:
            blew = True
            break
    assert blew


# --------------------------------------------------------------------------
# P13: wall viscous force (eq. 18) and the torque reduction, against the
# Stokes flow between concentric spheres (Re ~ 1e-3, no gravity, eq. 15)
# --------------------------------------------------------------------------

def _couette(ora, dp, om_outer, om_inner, steps, rigid_start=False, **over):
    """Run the sphere Couette case; axial torques on the inner and outer
    sphere per step, per unit Stokes torque at unit angular speed."""
    import dataclasses
    c = cases.sphere_couette(dp=dp)
    b0, b1 = c.bodies
    vf = np.cross([0.0, 0.0, om_inner], c.xf) if rigid_start else np.zeros_like(c.xf)
    c = dataclasses.replace(c, bodies=[dataclasses.replace(b0, omega=om_outer),
                                       dataclasses.replace(b1, omega=om_inner)],
                            vf=np.ascontiguousarray(vf))
    s = ora.State(c, **over)
    R1, R2 = c.meta["R1"], c.meta["R2"]
    eta = c.params["rho0"] * c.params["nu"]
    tau = 8 * math.pi * eta * R1 ** 3 * R2 ** 3 / (R2 ** 3 - R1 ** 3)   # per unit angular speed
    t_in, t_out = [], []
    for _ in range(steps):
        r = s.step()
        t_in.append(r["bodies"][1]["torque_axis"] / tau)
        t_out.append(r["bodies"][0]["torque_axis"] / tau)
    return s, c, np.array(t_in), np.array(t_out)


def _omega_profile_error(s, c, om_outer, om_inner, dp):
    """Largest deviation of the fluid's angular speed from the Stokes profile,
    per unit driving speed, over particles at least dp from either wall."""
    R1, R2 = c.meta["R1"], c.meta["R2"]
    x, v = s.x, s.v
    r = np.linalg.norm(x, axis=1)
    rc = np.hypot(x[:, 0], x[:, 1])
    om = (x[:, 0] * v[:, 1] - x[:, 1] * v[:, 0]) / np.maximum(rc ** 2, 1e-300)
    # Omega(r) = A + B / r^3 with Omega(R1) = om_inner, Omega(R2) = om_outer
    B = (om_inner - om_outer) * R1 ** 3 * R2 ** 3 / (R2 ** 3 - R1 ** 3)
    A = om_outer - B / R2 ** 3
    sel = (rc > 0.3 * r) & (r > R1 + dp) & (r < R2 - dp)
    return np.max(np.abs(om[sel] - (A + B / r[sel] ** 3))) / max(abs(om_inner), abs(om_outer))


@pytest.mark.parametrize("driven", ["inner", "outer"])
def test_stokes_torque_on_the_wall_at_rest(ora, driven):
    """Eq. 18 with the generalized wall's no-slip dummy velocity (Section 2.5).

    One sphere turns at 1 rad/s, the other is held.  At steady state the
    torque on the sphere at rest is the Stokes torque
    8 pi eta omega R1^3 R2^3 / (R2^3 - R1^3) within 10 % at dp = 0.5 mm (ten
    particles across the gap; measured 2.4 %), with the sign of a driven
    body, and the angular speed of the fluid follows the Stokes profile
    Omega(r) = A + B/r^3 within 5 % of the driving speed.  The literal
    reading of eq. 18 (dummy particles at the body's velocity) slips: its
    profile is 20-25 % slow and its torque 15-25 % low.
    """
    om_o, om_i = (0.0, 1.0) if driven == "inner" else (1.0, 0.0)
    s, c, t_in, t_out = _couette(ora, 0.5e-3, om_o, om_i, 200)
    rest, turning = (t_out, t_in) if driven == "inner" else (t_in, t_out)
    assert abs(rest[-1] - 1.0) <= 0.10, rest[-1]          # dragged forward by the fluid
    assert abs(rest[-1] - rest[-20]) <= 1e-3 * abs(rest[-1])          # steady
    assert _omega_profile_error(s, c, om_o, om_i, 0.5e-3) <= 0.05
    assert turning[-1] < 0                                  # the driven body is resisted


def test_literal_wall_velocity_slips(ora):
    """The reading that was not taken: dummy particles at the body's own
    velocity in eq. 18 leave the fluid slipping at the wall."""
    s, c, _, t_out = _couette(ora, 1.0e-3, 0.0, 1.0, 60, wall_visc=1)
    assert t_out[-1] < 0.85
    assert _omega_profile_error(s, c, 0.0, 1.0, 1.0e-3) > 0.08      # measured 0.10
    s, c, _, t_out = _couette(ora, 1.0e-3, 0.0, 1.0, 60)
    assert abs(t_out[-1] - 1.0) <= 0.10
    assert _omega_profile_error(s, c, 0.0, 1.0, 1.0e-3) <= 0.05


def test_torque_on_a_turning_wall_is_stokes_plus_its_corotation_reading(ora):
    """The pairwise reduction (torque = sum of (x_w - c) x (-f_iw)) of the
    non-central viscous pair forces of eq. 10 and 18 reads a torque on a body
    even when fluid and body co-rotate rigidly, where the exact torque is zero.
    In the Stokes regime the flow is linear in the wall speeds, so the torque
    read on the turning inner sphere equals the torque read under rigid
    co-rotation minus the torque read on it, at rest, when the outer sphere
    turns instead (the Stokes value): checked to 0.5 % of the Stokes torque.
    Rigid co-rotation keeps the fluid turning rigidly within 5 %."""
    _, _, i_in, i_out = _couette(ora, 1.0e-3, 0.0, 1.0, 60)           # inner turns
    _, _, o_in, o_out = _couette(ora, 1.0e-3, 1.0, 0.0, 60)           # outer turns
    s, c, r_in, r_out = _couette(ora, 1.0e-3, 1.0, 1.0, 60, rigid_start=True)
    assert abs(i_in[-1] - (r_in[-1] - o_in[-1])) <= 5e-3
    assert abs(i_out[-1] - (r_out[-1] - o_out[-1])) <= 5e-3
    assert abs(o_in[-1] - 1.0) <= 0.10          # the held inner sphere reads Stokes
    assert abs(i_out[-1] - 1.0) <= 0.10         # and so does the held outer one
    assert _omega_profile_error(s, c, 1.0, 1.0, 1.0e-3) <= 0.05
