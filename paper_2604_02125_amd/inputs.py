"""Seeded synthetic inputs for the cRKFR workloads.

This module holds no part of the numerical method: it only samples initial
conditions at given nodal coordinates and converts primitive to conserved
variables.  Both the GPU path and the CPU oracle take their inputs from here;
the reference nodes ``xi`` on [0, 1] are passed in by the caller, so each side
can use its own Gauss-Lobatto nodes.

Array layout: ``u[v, e, node]`` with element ``e = ey*nx + ex`` and node
``j*(N+1) + i`` (x index fastest).

Workloads (the paper's own test cases, Section 4, and their synthetic
stand-ins):
  * ``density_wave_1d``: smooth density wave, 1D Euler (convergence study);
  * ``kelvin_helmholtz``: Kelvin-Helmholtz instability on [-1,1]^2 (Section 4.2;
    the density base value is a parameter, see ``rho_base``);
  * ``orszag_tang``: Orszag-Tang vortex for ideal GLM-MHD on [0,1]^2;
  * ``random_fourier``: smooth random periodic Euler states for the batch of
    independent problems;
  * ``richtmyer_meshkov``: the Richtmyer-Meshkov initial data of Section 4.3.
"""
from __future__ import annotations

import numpy as np


def node_coords_1d(nx, x0, x1, xi):
    dx = (x1 - x0) / nx
    e = np.arange(nx)[:, None]
    return x0 + (e + np.asarray(xi)[None, :]) * dx


def node_coords_2d(nx, ny, x0, x1, y0, y1, xi):
    """X, Y of shape [E, (N+1)^2]."""
    xi = np.asarray(xi)
    n = xi.size
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    ex = np.arange(nx)
    ey = np.arange(ny)
    # node (i, j) -> index j*n + i
    Xi = np.tile(xi, n)            # xi_i for index j*n+i
    Yj = np.repeat(xi, n)          # xi_j
    X = x0 + (ex[None, :, None] + Xi[None, None, :]) * dx   # [1, nx, np]
    Y = y0 + (ey[:, None, None] + Yj[None, None, :]) * dy   # [ny, 1, np]
    X = np.broadcast_to(X, (ny, nx, n * n)).reshape(ny * nx, n * n)
    Y = np.broadcast_to(Y, (ny, nx, n * n)).reshape(ny * nx, n * n)
    return X.copy(), Y.copy()


def euler_conserved(rho, vels, p, gamma):
    """Stack (rho, rho v_d ..., E) into u[v, e, node]."""
    ke = sum(0.5 * rho * v * v for v in vels)
    return np.stack([rho] + [rho * v for v in vels] + [p / (gamma - 1.0) + ke]).astype(np.float64)


def density_wave_1d(nx, xi, gamma=1.4, x0=0.0, x1=1.0, t=0.0):
    """rho = 1 + 0.98 sin(2 pi (x - 0.1 t)), v = 0.1, p = 20 on a periodic line."""
    X = node_coords_1d(nx, x0, x1, xi)
    rho = 1.0 + 0.98 * np.sin(2 * np.pi * (X - 0.1 * t))
    return euler_conserved(rho, [np.full_like(X, 0.1)], np.full_like(X, 20.0), gamma)


def density_wave_2d(nx, ny, xi, gamma=1.4, t=0.0):
    """rho = 1 + 0.5 sin(2 pi (x + y - 0.3 t)), v = (0.1, 0.2), p = 20 on [0,1]^2."""
    X, Y = node_coords_2d(nx, ny, 0.0, 1.0, 0.0, 1.0, xi)
    rho = 1.0 + 0.5 * np.sin(2 * np.pi * (X + Y - 0.3 * t))
    return euler_conserved(rho, [np.full_like(X, 0.1), np.full_like(X, 0.2)], np.full_like(X, 20.0), gamma)


def kelvin_helmholtz(nx, ny, xi, gamma=1.4, rho_base=0.5, v2_modes=None):
    """B = tanh(15 y + 7.5) - tanh(15 y - 7.5); rho = rho_base + 3B/4,
    v1 = (B - 1)/2, v2 = sin(2 pi x)/10, p = 1 on [-1,1]^2.

    ``v2_modes`` = [(c_k, k, phi_k), ...] replaces v2 by 0.1 * sum c_k sin(2 pi k x + phi_k)
    (seeded variants for generating training snapshots)."""
    X, Y = node_coords_2d(nx, ny, -1.0, 1.0, -1.0, 1.0, xi)
    B = np.tanh(15.0 * Y + 7.5) - np.tanh(15.0 * Y - 7.5)
    rho = rho_base + 0.75 * B
    v1 = 0.5 * (B - 1.0)
    if v2_modes is None:
        v2 = 0.1 * np.sin(2 * np.pi * X)
    else:
        v2 = 0.1 * sum(c * np.sin(2 * np.pi * k * X + ph) for c, k, ph in v2_modes)
    return euler_conserved(rho, [v1, v2], np.ones_like(X), gamma)


def khi_modes(seed):
    """Four random modes for the v2 perturbation, amplitudes normalised to sum 1."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, 4)
    c = c / c.sum()
    ph = rng.uniform(0.0, 2 * np.pi, 4)
    return [(c[k], k + 1, ph[k]) for k in range(4)]


def orszag_tang(nx, ny, xi, gamma=5.0 / 3.0):
    """rho = 25/(36 pi), p = 5/(12 pi), v = (-sin 2pi y, sin 2pi x, 0),
    B = (-sin 2pi y, sin 4pi x, 0)/sqrt(4 pi), psi = 0 on [0,1]^2.
    Conserved order (rho, rho v1, rho v2, rho v3, E, B1, B2, B3, psi)."""
    X, Y = node_coords_2d(nx, ny, 0.0, 1.0, 0.0, 1.0, xi)
    rho = np.full_like(X, 25.0 / (36.0 * np.pi))
    p = np.full_like(X, 5.0 / (12.0 * np.pi))
    v1, v2, v3 = -np.sin(2 * np.pi * Y), np.sin(2 * np.pi * X), np.zeros_like(X)
    s = 1.0 / np.sqrt(4 * np.pi)
    B1, B2, B3 = -np.sin(2 * np.pi * Y) * s, np.sin(4 * np.pi * X) * s, np.zeros_like(X)
    psi = np.zeros_like(X)
    E = p / (gamma - 1.0) + 0.5 * rho * (v1 ** 2 + v2 ** 2 + v3 ** 2) + 0.5 * (B1 ** 2 + B2 ** 2 + B3 ** 2) + 0.5 * psi ** 2
    return np.stack([rho, rho * v1, rho * v2, rho * v3, E, B1, B2, B3, psi]).astype(np.float64)


def _fourier_field(rng, X, Y, amp_max, mean):
    f = np.full_like(X, mean)
    for _ in range(4):
        A = rng.uniform(0.0, amp_max)
        kx, ky = rng.integers(1, 5), rng.integers(1, 5)
        ph = rng.uniform(0.0, 2 * np.pi)
        f = f + A * np.sin(2 * np.pi * (kx * X + ky * Y) + ph)
    return f


def random_fourier_problems(nprob, seed=20260402, n_range=(16, 96), degrees=(3, 4)):
    """Draw the sizes and degrees of ``nprob`` independent periodic problems on
    [0,1]^2: n ~ U{n_range}, N uniformly from ``degrees``, in problem order."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(nprob):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        N = int(degrees[int(rng.integers(0, len(degrees)))])
        specs.append((n, N))
    return specs, rng


def random_fourier_state(rng, n, xi, gamma=1.4):
    """rho, p = 1 + 4 random modes (amplitude <= 0.2, wavenumbers 1..4),
    v1, v2 = 4 random modes of amplitude <= 0.3 and zero mean."""
    X, Y = node_coords_2d(n, n, 0.0, 1.0, 0.0, 1.0, xi)
    rho = _fourier_field(rng, X, Y, 0.2, 1.0)
    p = _fourier_field(rng, X, Y, 0.2, 1.0)
    v1 = _fourier_field(rng, X, Y, 0.3, 0.0)
    v2 = _fourier_field(rng, X, Y, 0.3, 0.0)
    return euler_conserved(rho, [v1, v2], p, gamma)


def richtmyer_meshkov(nx, ny, xi, gamma=1.4):
    """Section 4.3: d_{a,b}(x) = a + (1 + tanh(2x))(b - a)/2,
    rho = d_{1,1/4}(y - (18 + 2 cos(6 pi x / 40))) + d_{3.22,0}(|y - 4| - 2),
    p = d_{4.9,1}(|y - 4| - 2), v = 0 on [0, 40/3] x [0, 40]."""
    X, Y = node_coords_2d(nx, ny, 0.0, 40.0 / 3.0, 0.0, 40.0, xi)

    def d(a, b, x):
        return a + (1.0 + np.tanh(2.0 * x)) * (b - a) / 2.0

    rho = d(1.0, 0.25, Y - (18.0 + 2.0 * np.cos(6 * np.pi * X / 40.0))) + d(3.22, 0.0, np.abs(Y - 4.0) - 2.0)
    p = d(4.9, 1.0, np.abs(Y - 4.0) - 2.0)
    return euler_conserved(rho, [np.zeros_like(X), np.zeros_like(X)], p, gamma)


def random_smooth_euler(nx, ny, xi, seed, gamma=1.4, dim=2, amp=0.2):
    """Generic seeded smooth positive Euler state (parity tests)."""
    rng = np.random.default_rng(seed)
    if dim == 1:
        X = node_coords_1d(nx, 0.0, 1.0, xi)
        Y = np.zeros_like(X)
    else:
        X, Y = node_coords_2d(nx, ny, 0.0, 1.0, 0.0, 1.0, xi)
    rho = _fourier_field(rng, X, Y, amp, 1.0)
    p = _fourier_field(rng, X, Y, amp, 1.0)
    vels = [_fourier_field(rng, X, Y, 1.5 * amp, 0.0) for _ in range(dim)]
    return euler_conserved(rho, vels, p, gamma)


def random_smooth_mhd(nx, ny, xi, seed, gamma=5.0 / 3.0, amp=0.2):
    rng = np.random.default_rng(seed)
    X, Y = node_coords_2d(nx, ny, 0.0, 1.0, 0.0, 1.0, xi)
    rho = _fourier_field(rng, X, Y, amp, 1.0)
    p = _fourier_field(rng, X, Y, amp, 1.0)
    v = [_fourier_field(rng, X, Y, 1.5 * amp, 0.0) for _ in range(3)]
    B = [_fourier_field(rng, X, Y, 1.5 * amp, 0.0) for _ in range(3)]
    psi = _fourier_field(rng, X, Y, 0.5 * amp, 0.0)
    E = p / (gamma - 1.0) + 0.5 * rho * sum(c * c for c in v) + 0.5 * sum(c * c for c in B) + 0.5 * psi ** 2
    return np.stack([rho, rho * v[0], rho * v[1], rho * v[2], E, B[0], B[1], B[2], psi]).astype(np.float64)


def perturb(u, seed, rel=1e-3):
    """Multiply by (1 + rel * U(-1,1)) noise: breaks symmetries, keeps positivity."""
    rng = np.random.default_rng(seed)
    return u * (1.0 + rel * rng.uniform(-1.0, 1.0, size=u.shape))
