"""Pins of the oracle's learned-indicator MLP (FP64): a hand-computed
forward pass, finite-difference gradients, and a closed-form Adam step."""
import math

import numpy as np


def test_mlp_forward_hand_computed(orc):
    # nin = 1, H = 1: W1=2, b1=-1, W2=3, b2=0.5, W3=-1, b3=0.25, x = 1
    # a1 = 1 -> h1 = 1; a2 = 3.5 -> h2 = 3.5; z = -3.25
    theta = np.array([2.0, -1.0, 3.0, 0.5, -1.0, 0.25])
    assert orc.mlp_nparams(1, 1) == 6
    z, a = orc.mlp_forward(1, 1, theta, np.array([[1.0], [0.2]]), 0.008)
    assert z[0] == -3.25
    assert abs(a[0] - 0.008 / (1 + math.exp(3.25))) < 1e-18
    # x = 0.2: a1 = -0.6 -> relu 0; a2 = 0.5; z = -0.25
    assert z[1] == -0.25


def test_mlp_gradient_finite_differences(orc):
    nin, H = 16, 8
    rng = np.random.default_rng(3)
    theta = rng.normal(scale=0.5, size=orc.mlp_nparams(nin, H))
    x = rng.uniform(0, 1, (20, nin))
    y = (rng.uniform(size=20) > 0.5).astype(float)
    loss, g = orc.mlp_loss_grad(nin, H, theta, x, y)
    # loss itself against the textbook BCE of sigmoid(z)
    z, _ = orc.mlp_forward(nin, H, theta, x, 1.0)
    s = 1 / (1 + np.exp(-z))
    assert abs(loss - np.mean(-y * np.log(s) - (1 - y) * np.log(1 - s))) < 1e-13
    for k in rng.choice(theta.size, 40, replace=False):
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (orc.mlp_loss_grad(nin, H, tp, x, y)[0] - orc.mlp_loss_grad(nin, H, tm, x, y)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * (1 + abs(g[k]))


def test_adam_first_step(orc):
    # from zero moments the bias-corrected first step is -lr * g / (|g| + eps)
    theta = np.array([1.0, -2.0, 0.5])
    m, v = np.zeros(3), np.zeros(3)
    g = np.array([0.3, -4.0, 0.0])
    orc.adam_step(theta, m, v, g, 0.01, 1)
    assert np.allclose(theta, [1.0 - 0.01 * 0.3 / (0.3 + 1e-8), -2.0 + 0.01 * 4.0 / (4.0 + 1e-8), 0.5], atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_labels_special_cases(orc):
    """Troubled-element labels: a constant state and its exact free-stream
    update are untroubled; an overshoot, an undershoot beyond the 1e-3
    band, a negative pressure and a NaN are each flagged in their element
    only."""
    prob = orc.Problem(dim=2, N=3, nx=4, ny=3)
    u = np.zeros(prob.shape)
    u[0], u[1], u[2], u[3] = 1.0, 0.1, 0.0, 2.5
    assert not orc.labels(prob, u, u.copy()).any()
    uh = u.copy()
    uh[0, 5, 3] = 1.0 + 0.5e-3                     # inside the band
    assert not orc.labels(prob, u, uh).any()
    uh[0, 5, 3] = 1.0 + 2e-3                       # density overshoot
    uh[3, 9, 0] = 0.1                              # pressure undershoot in element 9
    uh[3, 2, 7] = -1.0                             # negative pressure in element 2
    uh[1, 11, 1] = np.nan                          # non-finite in element 11
    lab = orc.labels(prob, u, uh)
    assert np.flatnonzero(lab).tolist() == [2, 5, 9, 11]
    # the bounds include the face neighbours: a value present in a neighbour is allowed
    u2 = u.copy()
    u2[0, 6] = 1.5                                 # element 6 is a face neighbour of 5 (4 x 3 mesh)
    uh2 = u2.copy()
    uh2[0, 5, 0] = 1.4
    assert orc.labels(prob, u2, uh2)[5] == 0.0
    uh2[0, 5, 0] = 1.6
    assert orc.labels(prob, u2, uh2)[5] == 1.0


def test_feature_transform(orc):
    f = np.array([1.0, 0.1, 1e-8, 1e-16, 1e-20, 0.0])
    assert np.allclose(orc.feature_transform(f), [1.0, 1 - 1 / 16, 0.5, 0.0, 0.0, 0.0], atol=1e-15)
