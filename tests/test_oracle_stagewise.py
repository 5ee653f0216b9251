"""Pins of the oracle's stage-wise non-conservative interface flux
(eq:bad.numflux.non.cons, with the factor 1/2 of eq:non.cons.num.flux.basic):
  F^{num,nc,+-} = sum_j b_j 1/2 B(u^{(j),+-}) (g(u^{(j),-}) + g(u^{(j),+})),
against the reduced form 1/2 B(u^{n,+-}) (g(U^-) + g(U^+)) that the paper
uses.  g is linear in u, so the two differ only through B evaluated at the
stage states instead of u^n:
  * with one stage (u^(1) = u^n, U = u^n) they are the same arithmetic;
  * a constant state is preserved by both;
  * per step they differ by dt * O(dt): halving dt divides the difference
    of the updates by about 4 (a dropped or doubled factor would leave an
    O(dt) difference, ratio 2)."""
import numpy as np

from paper_2604_02125_amd import inputs


def _mhd(orc, **kw):
    base = dict(dim=2, N=3, nx=5, ny=4, eq=orc.MHD, gamma=5.0 / 3.0, vol_flux=orc.VOL_DERIGS)
    base.update(kw)
    return orc.Problem(**base)


def test_one_stage_forms_coincide(orc):
    xi, _ = orc.gll(3)
    u = inputs.perturb(inputs.random_smooth_mhd(5, 4, xi, seed=12, amp=0.25), 13, 1e-2)
    red = _mhd(orc, A=orc.EULER1_A, b=orc.EULER1_B)
    stg = _mhd(orc, A=orc.EULER1_A, b=orc.EULER1_B, nc_stagewise=1)
    red.ch = stg.ch = orc.compute_ch(red, u)
    dt = orc.compute_dt(red, u)
    a, _ = orc.crk_step(red, u, dt)
    b, _ = orc.crk_step(stg, u, dt)
    assert np.array_equal(a, b)


def test_constant_state_preserved(orc):
    stg = _mhd(orc, N=4, nx=3, ny=3, nc_stagewise=1)
    g = 5.0 / 3.0
    rho, v, p, B, psi = 1.3, np.array([0.4, -0.7, 0.2]), 0.9, np.array([0.8, -0.5, 0.3]), 0.25
    u0 = np.array([rho, *(rho * v), p / (g - 1) + 0.5 * rho * v @ v + 0.5 * B @ B + 0.5 * psi ** 2, *B, psi])
    u = np.broadcast_to(u0[:, None, None], stg.shape).copy()
    stg.ch = orc.compute_ch(stg, u)
    u1, _ = orc.crk_step(stg, u, orc.compute_dt(stg, u))
    assert np.max(np.abs(u1 - u)) < 1e-14 * np.max(np.abs(u))


def test_difference_is_second_order_in_dt(orc):
    xi, _ = orc.gll(3)
    u = inputs.random_smooth_mhd(5, 4, xi, seed=14, amp=0.25)
    red = _mhd(orc)
    stg = _mhd(orc, nc_stagewise=1)
    red.ch = stg.ch = orc.compute_ch(red, u)
    dt = orc.compute_dt(red, u)
    diffs = []
    for h in (dt, dt / 2, dt / 4):
        a, _ = orc.crk_step(red, u, h)
        b, _ = orc.crk_step(stg, u, h)
        diffs.append(np.max(np.abs(a - b)))
    assert diffs[0] > 1e-10                 # the forms do differ
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, diffs
