"""Pins of the oracle's reference element (paper Section 2: GLL solution
points on [0,1], eq:diff.matrix, g2 correction functions) against closed
forms, exactness properties and the summation-by-parts identity."""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gll_closed_forms.txt")


def _golden():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            N, xs, ws = line.split("|")
            ev = lambda s: [eval(t, {"sqrt": math.sqrt}) for t in s.split(";")]  # noqa: E731
            rows[int(N)] = (np.array(ev(xs)), np.array(ev(ws)))
    return rows


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_closed_forms(orc, N):
    xi, w = orc.gll(N)
    gx, gw = _golden()[N]
    assert np.max(np.abs(xi - gx)) < 1e-15
    assert np.max(np.abs(w - gw)) < 1e-15


@pytest.mark.parametrize("N", range(1, 9))
def test_gll_quadrature_exactness(orc, N):
    # Lobatto quadrature with N+1 points integrates degree <= 2N-1 exactly on [0,1]
    xi, w = orc.gll(N)
    for k in range(2 * N):
        assert abs(np.sum(w * xi ** k) - 1.0 / (k + 1)) < 1e-14
    # ... and is not exact for degree 2N (guards against a Gauss rule by mistake)
    assert abs(np.sum(w * xi ** (2 * N)) - 1.0 / (2 * N + 1)) > 1e-11


@pytest.mark.parametrize("N", range(1, 9))
def test_diffmat_exact_on_polynomials(orc, N):
    xi, _ = orc.gll(N)
    D = orc.diffmat(N, xi)
    for k in range(N + 1):
        dk = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        assert np.max(np.abs(D @ xi ** k - dk)) < 1e-11 * (N + 1) ** 2
    assert np.max(np.abs(D.sum(axis=1))) < 1e-12          # constants have zero derivative
    assert abs(D[0, 0] + N * (N + 1) / 2.0) < 1e-12           # D_00 = -N(N+1)/2 on [0,1]


@pytest.mark.parametrize("N", range(1, 9))
def test_sbp_identity(orc, N):
    # Q = diag(w) D satisfies Q + Q^T = diag(-1, 0, ..., 0, 1)
    xi, w = orc.gll(N)
    Q = np.diag(w) @ orc.diffmat(N, xi)
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    assert np.max(np.abs(Q + Q.T - B)) < 1e-13


@pytest.mark.parametrize("N", range(1, 9))
def test_g2_lifting_on_gll(orc, N):
    # Huynh's g2 built from Radau polynomials has, at GLL nodes on [0,1],
    # g_L' = -delta_p0 / w_0 and g_R' = delta_pN / w_N (the lumped lifting).
    xi, w = orc.gll(N)
    gl, gr = orc.g2_derivatives(N, xi)
    el = np.zeros(N + 1)
    el[0] = -1.0 / w[0]
    er = np.zeros(N + 1)
    er[N] = 1.0 / w[N]
    assert np.max(np.abs(gl - el)) < 1e-11 * (N + 1) ** 2
    assert np.max(np.abs(gr - er)) < 1e-11 * (N + 1) ** 2


def _rk_error(A, b, h):
    # y' = y, y(0) = 1 over one step; exact e^h
    s = len(b)
    k = np.zeros(s)
    for i in range(s):
        k[i] = 1.0 + h * sum(A[i][j] * k[j] for j in range(i))
    return abs(1.0 + h * sum(b[i] * k[i] for i in range(s)) - math.exp(h))


@pytest.mark.parametrize("name,order", [("RK4", 4), ("RK5", 5)])
def test_butcher_tableau_order(orc, name, order):
    A, b = (orc.RK4_A, orc.RK4_B) if name == "RK4" else (orc.RK5_A, orc.RK5_B)
    assert abs(sum(b) - 1.0) < 1e-15
    # local error O(h^{p+1}): halving h divides it by about 2^{p+1}
    r = _rk_error(A, b, 0.2) / _rk_error(A, b, 0.1)
    assert 2 ** (order + 1) * 0.8 < r < 2 ** (order + 1) * 1.25
    # on a nonlinear scalar problem y' = -y^2 (exact y = 1/(1+t)), global order
    def solve(h):
        y = 1.0
        for _ in range(int(round(1.0 / h))):
            s = len(b)
            k = []
            for i in range(s):
                yi = y + h * sum(A[i][j] * k[j] for j in range(i))
                k.append(-yi * yi)
            y += h * sum(b[i] * k[i] for i in range(s))
        return abs(y - 0.5)
    rr = solve(0.1) / solve(0.05)
    assert rr > 2 ** order * 0.8
