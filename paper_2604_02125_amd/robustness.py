"""Robustness runs of the cRKFR scheme (Section 4): a flow is stepped with
the pipelined GPU step until a final time or until the state becomes
non-physical (crk_check: a non-finite value, or rho <= 0 or p <= 0), and the
time reached is reported.  The paper's claims are of this form: with the
EC or KEP volume flux and the blending limiter the Kelvin-Helmholtz run of
Section 4.2 lasts to t = 15, while the same scheme without them (the
central volume flux, which recovers the plain FR derivative) stops at about
t = 4; the Richtmyer-Meshkov run of Section 4.3 lasts to t = 30 with the
EC/KEP fluxes and stops at about t = 8.7 without.

Every step of the method runs in the library; this module only drives the
time loop and reads dt back to accumulate the simulated time.
"""
from __future__ import annotations

import math

from . import crk, inputs


def run_until(solver, u0, t_end, check_every=100, max_steps=10_000_000):
    """Step u0 (host array) with the pipelined step until t >= t_end or a
    check fails.  Returns a dict: t reached, steps, whether it failed, the
    status and first bad element of the failing check, and the final
    minimum density and pressure."""
    import torch
    u = [torch.tensor(u0, dtype=solver.dtype, device=solver.device), solver.new_state()]
    dt = solver.new_dt()
    solver.prepare(u[0], dt)
    t, n = 0.0, 0
    status, first_bad = crk.OK, -1
    while t < t_end and n < max_steps:
        h = float(dt[0].item())
        if not math.isfinite(h) or h <= 0.0:
            status = crk.ERR_NOT_FINITE
            break
        solver.advance(u[n % 2], u[(n + 1) % 2], dt)
        t += h
        n += 1
        if n % check_every == 0 or t >= t_end:
            rc, first_bad, _ = solver.check(u[n % 2])
            if rc != crk.OK:
                status = rc
                break
    rc, fb, d = solver.check(u[n % 2])
    M = solver.shape[0]
    return {"t": t, "steps": n, "failed": status != crk.OK,
            "status": {crk.OK: "ok", crk.ERR_NOT_FINITE: "not finite",
                       crk.ERR_NONPHYSICAL: "non-physical"}.get(status, str(status)),
            "first_bad_element": int(first_bad), "min_rho": float(d[M + 1]), "min_p": float(d[M + 2])}


def khi_crash_study(fluxes=(crk.VOL_CENTRAL, crk.VOL_KG, crk.VOL_RANOCHA), n=64, t_end=15.0, alpha_max=0.008,
                    rho_base=0.25, precision=crk.FP64, check_every=100):
    """Section 4.2: compressible Euler Kelvin-Helmholtz instability on
    [-1,1]^2 periodic, n x n elements of degree 3, blending limiter with
    alpha_max, the paper's density rho = rho_base + 3B/4 (rho_base = 1/4),
    run to t_end once per volume flux."""
    names = {crk.VOL_CENTRAL: "central", crk.VOL_KG: "kennedy_gruber", crk.VOL_RANOCHA: "ranocha"}
    out = {}
    for f in fluxes:
        s = crk.Solver(dim=2, nx=n, ny=n, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, degree=3, precision=precision,
                       volume_flux=f, cfl=0.4, limiter=crk.LIM_BLEND, alpha_max=alpha_max, alpha_min=1e-3)
        xi, _, _ = crk.reference_element(3)
        u0 = inputs.kelvin_helmholtz(n, n, xi, rho_base=rho_base)
        out[names[f]] = run_until(s, u0, t_end, check_every=check_every)
    return out


def rmi_crash_study(fluxes=(crk.VOL_CENTRAL, crk.VOL_KG, crk.VOL_RANOCHA), nx=32, ny=96, t_end=30.0,
                    alpha_max=0.001, precision=crk.FP64, check_every=100):
    """Section 4.3: compressible Euler Richtmyer-Meshkov instability on
    [0, 40/3] x [0, 40], nx x ny elements of degree 3, blending limiter with
    alpha_max, reflective walls on all four sides (the paper gives no
    boundary conditions; the initial state is mirror-symmetric about the
    vertical walls, so there they agree with a periodic continuation), run
    to t_end once per volume flux."""
    names = {crk.VOL_CENTRAL: "central", crk.VOL_KG: "kennedy_gruber", crk.VOL_RANOCHA: "ranocha"}
    out = {}
    for f in fluxes:
        s = crk.Solver(dim=2, nx=nx, ny=ny, x0=0.0, x1=40.0 / 3.0, y0=0.0, y1=40.0, degree=3, precision=precision,
                       volume_flux=f, cfl=0.4, limiter=crk.LIM_BLEND, alpha_max=alpha_max, alpha_min=1e-3,
                       boundary=(crk.BC_WALL, crk.BC_WALL))
        xi, _, _ = crk.reference_element(3)
        u0 = inputs.richtmyer_meshkov(nx, ny, xi)
        out[names[f]] = run_until(s, u0, t_end, check_every=check_every)
    return out
