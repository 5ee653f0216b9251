"""Pins of the oracle's reflective walls (the reading taken for the
Richtmyer-Meshkov test of Section 4.3, whose boundary conditions the paper
does not state).  Beyond a wall lies the mirror image of the element, so a
walled mesh must reproduce, to rounding, the half of a periodic mesh twice
as long whose state is mirror-symmetric about the wall: this fixes every
component of the wall flux (mass, both momenta, energy), the Rusanov speed
and the blending coefficient across the wall.  Further: mass and energy are
conserved in a closed box, and a gas at rest stays at rest."""
import numpy as np
import pytest

from paper_2604_02125_amd import inputs


def _state(orc, prob, seed, amp=0.15):
    """A smooth positive state on the walled mesh whose mirror images across
    every wall continue it smoothly: rho, p and the tangential velocity are
    sums of cos(pi k x / L) in the walled direction (even about both ends),
    the normal velocity of sin(pi k x / L) (odd); periodic directions take
    full sine/cosine modes."""
    rng = np.random.default_rng(seed)
    xi, _ = orc.gll(prob.N)
    if prob.dim == 1:
        X = inputs.node_coords_1d(prob.nx, prob.x0, prob.x1, xi)
        Y = np.zeros_like(X)
    else:
        X, Y = inputs.node_coords_2d(prob.nx, prob.ny, prob.x0, prob.x1, prob.y0, prob.y1, xi)
    L = [prob.x1 - prob.x0, prob.y1 - prob.y0]
    C = [(X - prob.x0) / L[0], (Y - prob.y0) / L[1]]

    def field(mean, odd_dir=None):
        f = np.full_like(X, mean)
        for _ in range(3):
            a = rng.uniform(-amp, amp)
            term = np.ones_like(X)
            for d in range(prob.dim):
                k = rng.integers(1, 4)
                if prob.bc[d] == orc.BC_WALL:
                    term = term * (np.sin(np.pi * k * C[d]) if d == odd_dir else np.cos(np.pi * k * C[d]))
                else:
                    term = term * np.cos(2 * np.pi * k * C[d] + rng.uniform(0, 2 * np.pi))
            f = f + a * term
        return f
    rho, p = field(1.0), field(1.0)
    vel = [field(0.0, odd_dir=d) for d in range(prob.dim)]
    return inputs.euler_conserved(rho, vel, p, prob.gamma)


def _mirror_periodic(orc, prob, u, d):
    """The periodic mesh twice as long in direction d holding u and its
    mirror image (node order reversed along d, momentum d negated)."""
    n1 = prob.N + 1
    nx, ny = prob.nx, (prob.ny if prob.dim == 2 else 1)
    M = u.shape[0]
    if prob.dim == 1:
        m = u[:, ::-1, ::-1].copy()
        m[1 + d] *= -1.0
        return np.concatenate([u, m], axis=1)
    ue = u.reshape(M, ny, nx, n1, n1)           # [v, ey, ex, j, i]
    if d == 0:
        m = ue[:, :, ::-1, :, ::-1].copy()
        big = np.concatenate([ue, m], axis=2)
    else:
        m = ue[:, ::-1, :, ::-1, :].copy()
        big = np.concatenate([ue, m], axis=1)
    if d == 0:
        big[1 + d, :, nx:] *= -1.0
    else:
        big[1 + d, ny:] *= -1.0
    return big.reshape(M, -1, n1 * n1)


def _first_half_elements(prob, a, d):
    if prob.dim == 1:
        return a[:prob.nx]
    if d == 0:
        return a.reshape(prob.ny, 2 * prob.nx)[:, :prob.nx].ravel()
    return a.reshape(2 * prob.ny, prob.nx)[:prob.ny].ravel()


def _first_half(prob, big, d):
    n1 = prob.N + 1
    M = big.shape[0]
    if prob.dim == 1:
        return big[:, :prob.nx]
    nx, ny = prob.nx, prob.ny
    if d == 0:
        return big.reshape(M, ny, 2 * nx, n1 * n1)[:, :, :nx].reshape(M, -1, n1 * n1)
    return big.reshape(M, 2 * ny, nx, n1 * n1)[:, :ny].reshape(M, -1, n1 * n1)


CASES = [(1, 3, 2, 0, 0), (2, 3, 1, 0, 0), (2, 3, 1, 1, 1), (2, 4, 2, 1, 0), (2, 2, 1, 0, 1), (2, 1, 0, 0, 0)]


@pytest.mark.parametrize("dim,N,vol,d,lim", CASES)
def test_wall_equals_mirrored_periodic(orc, dim, N, vol, d, lim):
    bc = [orc.BC_PERIODIC, orc.BC_PERIODIC]
    bc[d] = orc.BC_WALL
    kw = dict(dim=dim, N=N, vol_flux=vol, nx=5, ny=4, x1=1.0, y1=0.8,
              limiter=orc.LIM_BLEND_MODAL if lim else orc.LIM_NONE)
    wall = orc.Problem(bc=tuple(bc), **kw)
    u = _state(orc, wall, seed=10 * N + d)
    if lim:
        # nodal noise, mirrored with the state, so that elements at the walls blend
        u = inputs.perturb(u, 3, 0.05)
    big_kw = dict(kw)
    if d == 0:
        big_kw.update(nx=2 * wall.nx, x1=2.0)
    else:
        big_kw.update(ny=2 * wall.ny, y1=1.6)
    per = orc.Problem(**big_kw)
    ub = _mirror_periodic(orc, wall, u, d)
    dt = orc.compute_dt(wall, u)
    assert abs(orc.compute_dt(per, ub) - dt) <= 1e-15 * dt
    uw, aw = orc.crk_step(wall, u, dt)
    up, ap = orc.crk_step(per, ub, dt)
    if lim:
        assert aw.max() > 0.0
        assert np.allclose(aw, _first_half_elements(wall, ap, d), rtol=1e-12, atol=1e-15)
    half = _first_half(wall, up, d)
    scale = np.max(np.abs(u), axis=(1, 2))[:, None, None]
    assert np.max(np.abs(uw - half) / scale) < 1e-13
    assert np.max(np.abs(uw - u) / scale) > 1e-6             # the step did something
    # and the semi-discrete operator beyond a wall sees the mirror image as well
    rw = orc.fr_rhs(wall, u)
    rp = _first_half(wall, orc.fr_rhs(per, ub), d)
    rs = np.max(np.abs(rp), axis=(1, 2))[:, None, None] + 1e-300
    assert np.max(np.abs(rw - rp) / rs) < 1e-12


@pytest.mark.parametrize("lim", [0, 1])
def test_closed_box_conserves_mass_and_energy(orc, lim):
    prob = orc.Problem(dim=2, N=3, nx=6, ny=9, x1=1.0, y1=1.5, vol_flux=orc.VOL_KG,
                       bc=(orc.BC_WALL, orc.BC_WALL), limiter=lim)
    u = inputs.perturb(_state(orc, prob, seed=5), 9, 0.05)
    t0 = orc.diagnostics(prob, u)["totals"]
    for _ in range(3):
        u, a = orc.crk_step(prob, u, orc.compute_dt(prob, u))
    t1 = orc.diagnostics(prob, u)["totals"]
    for v in (0, 3):
        assert abs(t1[v] - t0[v]) < 1e-14 * abs(t0[v])
    # the walls push: the momenta change
    assert max(abs(t1[1] - t0[1]), abs(t1[2] - t0[2])) > 1e-8
    if lim:
        assert a.max() > 0.0


def test_gas_at_rest_stays_at_rest(orc):
    for dim in (1, 2):
        prob = orc.Problem(dim=dim, N=3, nx=4, ny=3, vol_flux=orc.VOL_RANOCHA, bc=(orc.BC_WALL, orc.BC_WALL),
                           limiter=orc.LIM_BLEND_GIVEN)
        u = np.zeros(prob.shape)
        u[0] = 1.3
        u[dim + 1] = 0.9 / 0.4
        un, _ = orc.crk_step(prob, u, orc.compute_dt(prob, u), np.full(prob.nelem, 0.5))
        assert np.max(np.abs(un - u)) < 1e-15


def test_walls_are_euler_only(orc):
    prob = orc.Problem(dim=2, N=3, nx=3, ny=3, eq=orc.MHD, gamma=5 / 3, vol_flux=orc.VOL_DERIGS,
                       bc=(orc.BC_WALL, orc.BC_PERIODIC))
    with pytest.raises(ValueError):
        orc.crk_step(prob, np.ones(prob.shape), 1e-3)


def test_richtmyer_meshkov_initial_steps(orc):
    """Section 4.3's initial condition on a coarse version of its mesh
    (8 x 24 elements on [0, 40/3] x [0, 40], walls all round, Kennedy-Gruber,
    blending with alpha_max = 0.001): admissible and conservative."""
    prob = orc.Problem(dim=2, N=3, nx=8, ny=24, x1=40.0 / 3.0, y1=40.0, vol_flux=orc.VOL_KG,
                       limiter=orc.LIM_BLEND_MODAL, alpha_max=0.001, bc=(orc.BC_WALL, orc.BC_WALL))
    xi, _ = orc.gll(3)
    u = inputs.richtmyer_meshkov(8, 24, xi)
    t0 = orc.diagnostics(prob, u)["totals"]
    for _ in range(5):
        u, a = orc.crk_step(prob, u, orc.compute_dt(prob, u))
    d = orc.diagnostics(prob, u)
    assert d["first_bad"] == -1 and d["min_p"] > 0.5
    assert abs(d["totals"][0] - t0[0]) < 1e-14 * t0[0] and abs(d["totals"][3] - t0[3]) < 1e-14 * t0[3]
    assert a.max() > 0.0
