"""Pins of the oracle's GLM-MHD paths that the flux tests do not reach.

* The reduced-communication non-conservative interface flux
  1/2 B(u^{n,+-}) (g(U^-) + g(U^+)) of Section 2 (built from
  eq:non.cons.num.flux.basic; the factor 1/2 is the reading that makes the
  correction vanish for equal traces): a constant state with a normal field
  and a cleaning variable (so that B(u) g(u) != 0) must be preserved by the
  whole cRKFR step, and the semi-discrete operator with the entropy-
  conservative flux on the faces as well must produce no entropy on a
  periodic mesh (Rusanov faces: a negative rate).  Both fail when the factor
  1/2 is dropped.
* The fast magnetosonic speed for a field at any angle: c_f^2 is the larger
  root of c^4 - (a^2 + b^2) c^2 + a^2 b_d^2 = 0 (b = |B|/sqrt(rho),
  b_d = B_d/sqrt(rho)); for B perpendicular to d, c_f = sqrt(a^2 + b^2).
* The cleaning speed c_h of a state: the maximum over nodes and directions
  of |v_d| + c_f,d, here on a constant state with the closed forms above.
"""
import math

import numpy as np
import pytest

from paper_2604_02125_amd import inputs

G = 5.0 / 3.0


def _cons(rho, v, p, B, psi, g=G):
    v, B = np.asarray(v, float), np.asarray(B, float)
    E = p / (g - 1) + 0.5 * rho * v @ v + 0.5 * B @ B + 0.5 * psi * psi
    return np.array([rho, *(rho * v), E, *B, psi])


def _mhd(orc, **kw):
    base = dict(dim=2, eq=orc.MHD, gamma=G, vol_flux=orc.VOL_DERIGS)
    base.update(kw)
    return orc.Problem(**base)


@pytest.mark.parametrize("N,nx,ny", [(3, 5, 4), (4, 3, 3), (2, 4, 6)])
def test_mhd_constant_state_preserved(orc, N, nx, ny):
    prob = _mhd(orc, N=N, nx=nx, ny=ny)
    u0 = _cons(1.3, [0.4, -0.7, 0.2], 0.9, [0.8, -0.5, 0.3], 0.25)
    u = np.broadcast_to(u0[:, None, None], prob.shape).copy()
    prob.ch = orc.compute_ch(prob, u)
    # the non-conservative product of this state is not zero in either
    # direction, so an interface term that does not cancel would show
    for d in range(2):
        assert np.max(np.abs(orc.nc_two_point(prob, d, u0, u0))) > 0.1
    dt = orc.compute_dt(prob, u)
    u1, _ = orc.crk_step(prob, u, dt)
    assert np.max(np.abs(u1 - u)) < 1e-14 * np.max(np.abs(u))


def _entropy_rate(orc, prob, u, r):
    _, w = orc.gll(prob.N)
    wq = np.outer(w, w).ravel()
    rate = scale = 0.0
    for e in range(prob.nelem):
        for p in range(prob.nnode):
            wv = orc.entropy_vars(prob, u[:, e, p])
            rate += wq[p] * wv @ r[:, e, p]
            scale += wq[p] * np.abs(wv) @ np.abs(r[:, e, p])
    return rate, scale


@pytest.mark.parametrize("N", [3, 4])
def test_mhd_semidiscrete_ec_entropy_rate_zero(orc, N):
    """Derigs-form EC flux with the local Powell/GLM term in the volume, the
    same flux plus 1/2 B(u)(g^- + g^+) on the faces: dS/dt = 0 on a periodic
    mesh; Rusanov faces dissipate."""
    nx, ny = 4, 3
    xi, _ = orc.gll(N)
    prob = _mhd(orc, N=N, nx=nx, ny=ny)
    u = inputs.perturb(inputs.random_smooth_mhd(nx, ny, xi, seed=21, amp=0.25), 22, 1e-2)
    prob.ch = orc.compute_ch(prob, u)
    rate, scale = _entropy_rate(orc, prob, u, orc.fr_rhs(prob, u, orc.SURF_EC))
    assert abs(rate) < 1e-13 * scale, (rate, scale)
    rate, scale = _entropy_rate(orc, prob, u, orc.fr_rhs(prob, u, orc.SURF_RUSANOV))
    assert rate < -1e-6 * scale, (rate, scale)


def test_mhd_fast_speed_any_angle(orc):
    prob = _mhd(orc, ch=0.0)
    rng = np.random.default_rng(41)
    for _ in range(200):
        rho, p = rng.uniform(0.3, 2.0), rng.uniform(0.3, 2.0)
        v = rng.uniform(-1, 1, 3)
        B = rng.uniform(-1.5, 1.5, 3)
        u = _cons(rho, v, p, B, rng.uniform(-0.3, 0.3))
        a2 = G * p / rho
        b2 = B @ B / rho
        for d in range(2):
            cf = orc.wave_speed(prob, d, u) - abs(v[d])
            bd2 = B[d] ** 2 / rho
            # c_f^2 is a root of the characteristic quartic ...
            c2 = cf * cf
            assert abs(c2 * c2 - (a2 + b2) * c2 + a2 * bd2) < 1e-12 * (a2 + b2) ** 2
            # ... and the larger one: at least the mean of the two roots
            assert c2 >= 0.5 * (a2 + b2) * (1 - 1e-14)
    # field perpendicular to d: c_f = sqrt(a^2 + |B|^2/rho)
    rho, p = 1.7, 0.6
    u = _cons(rho, [0.3, -0.2, 0.1], p, [0.0, 0.9, -1.1], 0.1)
    want = math.sqrt(G * p / rho + (0.81 + 1.21) / rho)
    assert abs(orc.wave_speed(prob, 0, u) - 0.3 - want) < 1e-14 * want
    u = _cons(rho, [0.3, -0.2, 0.1], p, [0.7, 0.0, 0.4], 0.1)
    want = math.sqrt(G * p / rho + (0.49 + 0.16) / rho)
    assert abs(orc.wave_speed(prob, 1, u) - 0.2 - want) < 1e-14 * want


def test_mhd_cleaning_speed_of_constant_state(orc):
    prob = _mhd(orc, N=3, nx=3, ny=2)
    rho, p, Bx = 1.2, 0.8, 0.9
    v = [0.3, -0.5, 0.1]
    u0 = _cons(rho, v, p, [Bx, 0.0, 0.0], -0.2)
    u = np.broadcast_to(u0[:, None, None], prob.shape).copy()
    a = math.sqrt(G * p / rho)
    cfx = max(a, abs(Bx) / math.sqrt(rho))          # field along x
    cfy = math.sqrt(a * a + Bx * Bx / rho)          # field across y
    want = max(abs(v[0]) + cfx, abs(v[1]) + cfy)
    assert abs(orc.compute_ch(prob, u) - want) < 1e-14 * want
    # the Euler system has no cleaning speed
    assert orc.compute_ch(orc.Problem(dim=2, N=3, nx=2, ny=2), np.ones((4, 4, 16))) == 0.0
