"""Pins of the oracle's physics and two-point fluxes (paper Section 3,
eq:entropy.cons.flux.dev: f_S symmetric and consistent; EC fluxes satisfy
Tadmor's condition; KEP structure of the momentum flux)."""
import math

import numpy as np
import pytest


def _euler_state(rng, dim, gamma=1.4, scale=1.0):
    rho = rng.uniform(0.2, 3.0)
    v = rng.uniform(-1.5, 1.5, dim)
    p = rng.uniform(0.2, 3.0)
    return np.array([rho, *(rho * v), p / (gamma - 1) + 0.5 * rho * v @ v]) * scale


def _near(rng, u, sep):
    return u * (1.0 + sep * rng.uniform(-1, 1, u.size))


def _mhd_state(rng, gamma=5.0 / 3.0):
    rho = rng.uniform(0.3, 2.0)
    v = rng.uniform(-1.0, 1.0, 3)
    B = rng.uniform(-1.0, 1.0, 3)
    psi = rng.uniform(-0.3, 0.3)
    p = rng.uniform(0.3, 2.0)
    E = p / (gamma - 1) + 0.5 * rho * v @ v + 0.5 * B @ B + 0.5 * psi * psi
    return np.array([rho, *(rho * v), E, *B, psi])


def test_lnmean_against_log1p(orc):
    rng = np.random.default_rng(1)
    worst = 0.0
    for _ in range(4000):
        x = rng.uniform(0.1, 10.0)
        sep = 10.0 ** rng.uniform(-12, 0.0)
        y = x * (1.0 + sep * rng.choice([-0.9, 0.9]))
        exact = (x - y) / math.log1p((x - y) / y)      # ln x - ln y = log1p((x-y)/y)
        worst = max(worst, abs(orc.lnmean(x, y) - exact) / exact)
    assert worst < 5e-15
    assert orc.lnmean(2.0, 2.0) == 2.0
    # symmetric, and continuous across the series/log switch u = 1e-4
    for f in (0.0099, 0.01, 0.0101):
        x, y = 1.0 + f, 1.0 - f
        assert abs(orc.lnmean(x, y) - orc.lnmean(y, x)) < 1e-14
        assert abs(orc.lnmean(x, y) - (x - y) / (math.log1p(x - 1) - math.log1p(y - 1))) < 1e-14


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("vol", [0, 1, 2])
def test_consistency_and_symmetry(orc, dim, vol):
    prob = orc.Problem(dim=dim, vol_flux=vol)
    rng = np.random.default_rng(2)
    for _ in range(200):
        u, w = _euler_state(rng, dim), _euler_state(rng, dim)
        for d in range(dim):
            f = orc.phys_flux(prob, d, u)
            assert np.max(np.abs(orc.two_point(prob, d, u, u) - f)) < 1e-13 * (1 + np.max(np.abs(f)))
            assert np.max(np.abs(orc.two_point(prob, d, u, w) - orc.two_point(prob, d, w, u))) < 1e-13


def test_euler_physical_flux_closed_form(orc):
    # rho = 2, v = (3, -1), p = 5, gamma = 1.4: E = 5/0.4 + 0.5*2*10 = 22.5
    prob = orc.Problem(dim=2)
    u = np.array([2.0, 6.0, -2.0, 22.5])
    assert abs(orc.pressure(prob, u) - 5.0) < 1e-14
    assert np.allclose(orc.phys_flux(prob, 0, u), [6.0, 23.0, -6.0, 82.5], rtol=0, atol=1e-13)
    assert np.allclose(orc.phys_flux(prob, 1, u), [-2.0, -6.0, 7.0, -27.5], rtol=0, atol=1e-13)
    assert abs(orc.wave_speed(prob, 0, u) - (3.0 + math.sqrt(3.5))) < 1e-14


@pytest.mark.parametrize("dim", [1, 2])
def test_entropy_flux_compatibility(orc, dim):
    # continuous identity w(u)^T f'(u) = q'(u), checked by central differences;
    # pins the physical flux, the entropy variables and the entropy flux together
    prob = orc.Problem(dim=dim)
    rng = np.random.default_rng(3)
    for _ in range(30):
        u = _euler_state(rng, dim)
        w = orc.entropy_vars(prob, u)
        for d in range(dim):
            for c in range(u.size):
                h = 1e-6 * max(1.0, abs(u[c]))
                up, um = u.copy(), u.copy()
                up[c] += h
                um[c] -= h
                dfc = (orc.phys_flux(prob, d, up) - orc.phys_flux(prob, d, um)) / (2 * h)
                dqc = (orc.entropy_flux(prob, d, up) - orc.entropy_flux(prob, d, um)) / (2 * h)
                assert abs(w @ dfc - dqc) < 1e-7 * (1 + abs(dqc))
        # w = dS/du
        for c in range(u.size):
            h = 1e-6 * max(1.0, abs(u[c]))
            up, um = u.copy(), u.copy()
            up[c] += h
            um[c] -= h
            dS = (orc.entropy(prob, up) - orc.entropy(prob, um)) / (2 * h)
            assert abs(dS - w[c]) < 1e-7 * (1 + abs(w[c]))


def _tadmor_residual(orc, prob, d, uL, uR, theta=None):
    wL, wR = orc.entropy_vars(prob, uL), orc.entropy_vars(prob, uR)
    f = orc.two_point(prob, d, uL, uR)
    pL, pR = orc.flux_potential(prob, d, uL), orc.flux_potential(prob, d, uR)
    lhs = (wL - wR) @ f
    rhs = pL - pR
    scale = (np.abs(wL) + np.abs(wR)) @ np.abs(f) + abs(pL) + abs(pR)
    if theta is not None:
        tL, tR, bL, bR = theta
        rhs += 0.5 * (tL + tR) * (bL - bR)
        scale += abs(0.5 * (tL + tR)) * (abs(bL) + abs(bR))
    return abs(lhs - rhs) / scale


@pytest.mark.parametrize("dim", [1, 2])
def test_tadmor_condition_ranocha(orc, dim):
    prob = orc.Problem(dim=dim, vol_flux=orc.VOL_RANOCHA)
    rng = np.random.default_rng(4)
    worst = 0.0
    for it in range(3000):
        uL = _euler_state(rng, dim)
        uR = _euler_state(rng, dim) if it % 2 == 0 else _near(rng, uL, 10.0 ** rng.uniform(-9, -1))
        for d in range(dim):
            worst = max(worst, _tadmor_residual(orc, prob, d, uL, uR))
    assert worst < 1e-13


@pytest.mark.parametrize("vol", [0, 1])
def test_tadmor_fails_for_non_ec_fluxes(orc, vol):
    # sensitivity of the pin above: central and Kennedy-Gruber are not EC
    prob = orc.Problem(dim=2, vol_flux=vol)
    rng = np.random.default_rng(5)
    res = [_tadmor_residual(orc, prob, 0, _euler_state(rng, 2), _euler_state(rng, 2)) for _ in range(50)]
    assert np.median(res) > 1e-4


@pytest.mark.parametrize("vol", [1, 2])
def test_kep_structure(orc, vol):
    # KEP: momentum flux = mass flux * mean velocity + a pressure mean
    prob = orc.Problem(dim=2, vol_flux=vol)
    rng = np.random.default_rng(6)
    for _ in range(100):
        uL, uR = _euler_state(rng, 2), _euler_state(rng, 2)
        vL, vR = uL[1:3] / uL[0], uR[1:3] / uR[0]
        pm = 0.5 * (orc.pressure(prob, uL) + orc.pressure(prob, uR))
        for d in range(2):
            f = orc.two_point(prob, d, uL, uR)
            for k in range(2):
                expect = f[0] * 0.5 * (vL[k] + vR[k]) + (pm if k == d else 0.0)
                assert abs(f[1 + k] - expect) < 1e-13 * (1 + abs(expect))


def test_kennedy_gruber_closed_form(orc):
    # uL: rho=1, v=(1,0), p=1; uR: rho=3, v=(-1,2), p=2; gamma=1.4
    prob = orc.Problem(dim=2, vol_flux=orc.VOL_KG)
    g = 1.4
    uL = np.array([1.0, 1.0, 0.0, 1 / (g - 1) + 0.5])
    uR = np.array([3.0, -3.0, 6.0, 2 / (g - 1) + 0.5 * 3 * 5])
    eL, eR = uL[3] / 1.0, uR[3] / 3.0
    rho, v1, v2, p, e = 2.0, 0.0, 1.0, 1.5, 0.5 * (eL + eR)
    fx = orc.two_point(prob, 0, uL, uR)
    assert np.allclose(fx, [rho * v1, rho * v1 * v1 + p, rho * v1 * v2, (rho * e + p) * v1], atol=1e-14)
    fy = orc.two_point(prob, 1, uL, uR)
    assert np.allclose(fy, [rho * v2, rho * v2 * v1, rho * v2 * v2 + p, (rho * e + p) * v2], atol=1e-14)


# ---------------------------------------------------------------- GLM-MHD
def _mhd_prob(orc, ch=0.7):
    return orc.Problem(dim=2, eq=orc.MHD, gamma=5.0 / 3.0, vol_flux=orc.VOL_DERIGS, ch=ch)


def _theta(orc, prob, u, d):
    rho = u[0]
    v = u[1:4] / rho
    B = u[5:8]
    p = orc.pressure(prob, u)
    return rho / p * (v @ B), u[5 + d]


def test_mhd_consistency_symmetry(orc):
    prob = _mhd_prob(orc)
    rng = np.random.default_rng(7)
    for _ in range(200):
        u, w = _mhd_state(rng), _mhd_state(rng)
        for d in range(2):
            f = orc.phys_flux(prob, d, u)
            assert np.max(np.abs(orc.two_point(prob, d, u, u) - f)) < 1e-13 * (1 + np.max(np.abs(f)))
            assert np.max(np.abs(orc.two_point(prob, d, u, w) - orc.two_point(prob, d, w, u))) < 1e-13


def test_mhd_entropy_flux_compatibility(orc):
    # w^T f'(u) + theta dB_d/du = q'(u): the Powell term phi_P dB_d/dx with
    # theta = w.phi_P = (rho/p) v.B; the GLM term has w.phi_G = 0
    prob = _mhd_prob(orc)
    rng = np.random.default_rng(8)
    for _ in range(20):
        u = _mhd_state(rng)
        w = orc.entropy_vars(prob, u)
        for d in range(2):
            th, _ = _theta(orc, prob, u, d)
            for c in range(9):
                h = 1e-6 * max(1.0, abs(u[c]))
                up, um = u.copy(), u.copy()
                up[c] += h
                um[c] -= h
                dfc = (orc.phys_flux(prob, d, up) - orc.phys_flux(prob, d, um)) / (2 * h)
                dqc = (orc.entropy_flux(prob, d, up) - orc.entropy_flux(prob, d, um)) / (2 * h)
                lhs = w @ dfc + (th if c == 5 + d else 0.0)
                assert abs(lhs - dqc) < 1e-7 * (1 + abs(dqc))
            # phi_G is orthogonal to w
            phiG = orc.nc_two_point(prob, d, u, np.r_[np.zeros(5 + d), 0.0, np.zeros(2 - d), 1.0])
            assert abs(w @ phiG) < 1e-13 * (1 + np.max(np.abs(phiG)))


def test_mhd_generalised_tadmor(orc):
    # [[w]].f* = [[psi]] + {{theta}} [[B_d]]
    prob = _mhd_prob(orc)
    rng = np.random.default_rng(9)
    worst = 0.0
    for it in range(2000):
        uL = _mhd_state(rng)
        uR = _mhd_state(rng) if it % 2 == 0 else _near(rng, uL, 10.0 ** rng.uniform(-9, -1))
        for d in range(2):
            tL, bL = _theta(orc, prob, uL, d)
            tR, bR = _theta(orc, prob, uR, d)
            worst = max(worst, _tadmor_residual(orc, prob, d, uL, uR, (tL, tR, bL, bR)))
    assert worst < 1e-12


def test_mhd_central_fails_generalised_tadmor(orc):
    prob = orc.Problem(dim=2, eq=orc.MHD, gamma=5.0 / 3.0, vol_flux=orc.VOL_CENTRAL, ch=0.7)
    rng = np.random.default_rng(10)
    res = []
    for _ in range(50):
        uL, uR = _mhd_state(rng), _mhd_state(rng)
        tL, bL = _theta(orc, prob, uL, 0)
        tR, bR = _theta(orc, prob, uR, 0)
        res.append(_tadmor_residual(orc, prob, 0, uL, uR, (tL, tR, bL, bR)))
    assert np.median(res) > 1e-4


def test_mhd_fast_speed_reduces_to_sound_speed(orc):
    # B = 0: c_f = sqrt(gamma p / rho); B along d only: c_f = max(a, |B_d|/sqrt(rho))
    prob = _mhd_prob(orc, ch=0.0)
    g = 5.0 / 3.0
    rho, p = 2.0, 3.0
    u = np.array([rho, 0, 0, 0, p / (g - 1), 0, 0, 0, 0.0])
    assert abs(orc.wave_speed(prob, 0, u) - math.sqrt(g * p / rho)) < 1e-14
    u2 = u.copy()
    u2[5] = 4.0
    u2[4] += 0.5 * 16.0
    assert abs(orc.wave_speed(prob, 0, u2) - max(math.sqrt(g * p / rho), 4.0 / math.sqrt(rho))) < 1e-13
    # with cleaning speed larger than the fast speed, lambda = c_h
    prob2 = _mhd_prob(orc, ch=10.0)
    assert orc.wave_speed(prob2, 0, u) == 10.0
