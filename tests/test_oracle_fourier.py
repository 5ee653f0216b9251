"""Fourier pin of the oracle's cRKFR step (Section 2): for linear advection
u_t + a u_x = 0 the step is a linear map, and a Fourier mode exp(i k x) on a
periodic mesh of equal elements is multiplied, element by element, by an
(N+1) x (N+1) amplification matrix that follows from the scheme's
definition alone:
  inner stages     u^(i) = u^n - (a dt/dx) sum_j a_ij D u^(j)   (volume term only),
  time averages    U = sum_i b_i u^(i),   V = (a/dx) D U,   F = a U at the faces,
  interface flux   F* = 1/2 a (U^- + U^+) - 1/2 lambda (U^+ - U^-)     (eq:numflux.cons),
  update           u^{n+1} = u^n - dt V - (dt/dx) [ (F*_R - F_N)/w_N at xi = 1,
                                                   -(F*_L - F_0)/w_0 at xi = 0 ]
(g2 correction on GLL points).  The density of a 1D Euler state with
constant velocity v and pressure p and a small density wave of amplitude eps
advances by exactly this map with a = v and lambda = |v| + c (the sound
speed of the base state), up to O(eps^2): with v and p constant every
two-point flux is linear in rho in the density component, and the Rusanov
speed varies only at O(eps).  The amplification matrix is built here with
numpy only (GLL points from the Legendre polynomial, the differentiation
matrix from the Lagrange basis), independently of the oracle; a dropped
stage coupling, a wrong weight or a sign error in the interface terms moves
the result by O(1) relative to eps."""
import numpy as np
import pytest
from numpy.polynomial import legendre as L

RK4_A = [[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1, 0]]
RK4_B = [1 / 6, 1 / 3, 1 / 3, 1 / 6]
RK5_A = [[0, 0, 0, 0, 0, 0], [1 / 4, 0, 0, 0, 0, 0], [1 / 8, 1 / 8, 0, 0, 0, 0], [0, -1 / 2, 1, 0, 0, 0],
         [3 / 16, 0, 0, 9 / 16, 0, 0], [-3 / 7, 2 / 7, 12 / 7, -12 / 7, 8 / 7, 0]]
RK5_B = [7 / 90, 0, 32 / 90, 12 / 90, 32 / 90, 7 / 90]


def gll01(N):
    """GLL nodes and weights on [0, 1]: the end points and the roots of
    P_N'; weights 1/(N(N+1) P_N(x)^2) on [-1, 1], halved."""
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    inner = np.sort(np.real(L.legroots(L.legder(cN)))) if N > 1 else np.array([])
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (N * (N + 1) * L.legval(x, cN) ** 2)
    return (x + 1.0) / 2.0, w / 2.0


def diffmat(xi):
    """D[p, q] = l_q'(xi_p) for the Lagrange basis on the nodes xi."""
    n = len(xi)
    D = np.zeros((n, n))
    for q in range(n):
        others = [xi[m] for m in range(n) if m != q]
        denom = np.prod([xi[q] - o for o in others])
        coef = np.poly(others) / denom            # l_q as a monomial polynomial
        D[:, q] = np.polyval(np.polyder(coef), xi)
    return D


def amplification(N, A, b, nu, lam_over_a, theta, plant=None):
    """u^{n+1}_e = G u^n_e for the mode u_e = exp(i theta e) phi.  plant:
    a deliberate mistake, for the test that the comparison detects it."""
    xi, w = gll01(N)
    D = diffmat(xi)
    I = np.eye(N + 1)
    S = len(b)
    P = []                                        # u^(i) = P_i u^n
    for i in range(S):
        Pi = I.astype(complex)
        for j in range(i):
            aij = A[i][j] if plant != "stage" else 0.0
            Pi = Pi - nu * aij * D @ P[j]
        P.append(Pi)
    T = sum(b[i] * P[i] for i in range(S))       # U = T u^n
    eN, e0 = np.zeros(N + 1), np.zeros(N + 1)
    eN[N], e0[0] = 1.0, 1.0
    # interface fluxes in units of a: F*_R = 1/2 (U_N + s U_0) - 1/2 lam (s U_0 - U_N), s = exp(i theta)
    s = np.exp(1j * theta)
    FR = 0.5 * (np.outer(eN, eN) + s * np.outer(eN, e0)) - 0.5 * lam_over_a * (s * np.outer(eN, e0) - np.outer(eN, eN))
    FL = 0.5 * (np.outer(e0, eN) / s + np.outer(e0, e0)) - 0.5 * lam_over_a * (np.outer(e0, e0) - np.outer(e0, eN) / s)
    # rows: FR @ U gives F*_R in row N, FL @ U gives F*_L in row 0
    sl = -1.0 if plant == "left_sign" else 1.0
    corr = (FR - np.outer(eN, eN)) / w[N] - sl * (FL - np.outer(e0, e0)) / w[0]
    if plant == "no_upwind":
        corr = (FR + 0.5 * lam_over_a * (s * np.outer(eN, e0) - np.outer(eN, eN)) - np.outer(eN, eN)) / w[N] \
            - (FL + 0.5 * lam_over_a * (np.outer(e0, e0) - np.outer(e0, eN) / s) - np.outer(e0, e0)) / w[0]
    return I - nu * (D + corr) @ T


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("vol", [1, 2])
def test_density_wave_follows_the_amplification_matrix(orc, N, vol):
    nx, gamma, rho0, v, p0, eps = 10, 1.4, 1.0, 0.7, 0.9, 1e-7
    A, b = (RK5_A, RK5_B) if N >= 4 else (RK4_A, RK4_B)
    prob = orc.Problem(dim=1, nx=nx, N=N, vol_flux=vol, gamma=gamma)
    xi, _ = gll01(N)
    dx = 1.0 / nx
    c0 = np.sqrt(gamma * p0 / rho0)
    lam = abs(v) + c0
    worst = 0.0
    for m in (1, 2, 3):
        k = 2.0 * np.pi * m
        x = (np.arange(nx)[:, None] + xi[None, :]) * dx          # [e, p]
        rho = rho0 + eps * np.cos(k * x)
        u = np.zeros(prob.shape)
        u[0] = rho
        u[1] = rho * v
        u[2] = p0 / (gamma - 1.0) + 0.5 * rho * v * v
        dt = 0.5 * orc.compute_dt(prob, u)
        un, _ = orc.crk_step(prob, u, dt)
        G = amplification(N, A, b, v * dt / dx, lam / v, k * dx)
        phi = np.exp(1j * k * x)                                   # [e, p]
        pred = rho0 + eps * np.real(phi @ G.T)
        err = np.max(np.abs(un[0] - pred)) / eps
        # the mode really moved: the prediction differs from the input at O(eps)
        assert np.max(np.abs(pred - rho)) / eps > 1e-3
        # velocity and pressure stay constant
        assert np.max(np.abs(un[1] / un[0] - v)) < 1e-12
        worst = max(worst, err)
    assert worst < 1e-6, worst


@pytest.mark.parametrize("plant", ["stage", "left_sign", "no_upwind"])
def test_the_pin_sees_planted_mistakes(orc, plant):
    """The same comparison against a prediction with a planted mistake (inner
    stages left at u^n, the left-face correction with the wrong sign, no
    upwind part in the interface flux) misses by a hundred times the
    tolerance or more, on a less resolved mode (four waves on ten
    elements)."""
    N, nx, gamma, rho0, v, p0, eps = 3, 10, 1.4, 1.0, 0.7, 0.9, 1e-7
    prob = orc.Problem(dim=1, nx=nx, N=N, vol_flux=1, gamma=gamma)
    xi, _ = gll01(N)
    dx, k = 1.0 / nx, 2.0 * np.pi * 4
    x = (np.arange(nx)[:, None] + xi[None, :]) * dx
    rho = rho0 + eps * np.cos(k * x)
    u = np.zeros(prob.shape)
    u[0], u[1], u[2] = rho, rho * v, p0 / (gamma - 1.0) + 0.5 * rho * v * v
    dt = 0.5 * orc.compute_dt(prob, u)
    un, _ = orc.crk_step(prob, u, dt)
    lam = abs(v) + np.sqrt(gamma * p0 / rho0)
    phi = np.exp(1j * k * x)
    dev = {}
    for pl in (None, plant):
        G = amplification(N, RK4_A, RK4_B, v * dt / dx, lam / v, k * dx, plant=pl)
        dev[pl] = np.max(np.abs(un[0] - (rho0 + eps * np.real(phi @ G.T)))) / eps
    assert dev[None] < 1e-6 and dev[plant] > 1e-4, dev
