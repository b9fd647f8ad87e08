"""Pins of the FP64 allocator reference (oracle/budget.py) against things
other than itself: finite differences, closed forms of Adam and of the budget
rule, scipy's normal distribution, the pooled-MRL identity of the paper's
alignment proof, and a network small enough to evaluate by hand."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import budget as Bu
from oracle import oracle as O
from paper_2605_08048_amd import synth


def _net(seed):
    g = np.random.default_rng(seed)
    th = Bu.init_params(g, shift=g.normal(0, 1, Bu.NF), scale=g.uniform(0.5, 2.0, Bu.NF))
    P = Bu.unpack(th)
    P["b1"][:] = g.normal(0, 0.3, Bu.H1)   # non-zero biases so every term is exercised
    P["b2"][:] = g.normal(0, 0.3, Bu.H2)
    P["b3"][:] = g.normal(0, 0.3, Bu.NO)
    P["oshift"][:] = g.normal(0, 1, Bu.NO)
    P["oscale"][:] = g.uniform(0.2, 3.0, Bu.NO)
    X = g.normal(0, 1, (7, Bu.NF))
    T = g.normal(0, 1, (7, Bu.NO))
    return th, X, T


def test_layout():
    assert Bu.NPARAM == 12 + 12 + 2 + 2 + 64 * 12 + 64 + 64 * 64 + 64 + 2 * 64 + 2
    th = np.arange(Bu.NPARAM, dtype=np.float64)
    P = Bu.unpack(th)
    assert P["W1"][1, 0] == 28 + 12 and P["b3"][-1] == Bu.NPARAM - 1 and P["oscale"][0] == 26


def test_hand_network():
    """A network whose output can be written down: W1 copies feature 0 and its
    negative, W2 adds them after the ReLU (|x0|), W3 reads that and a bias."""
    th = np.zeros(Bu.NPARAM)
    P = Bu.unpack(th)
    P["shift"][:] = 1.0
    P["scale"][:] = 2.0
    P["oscale"][:] = 1.0
    P["W1"][0, 0], P["W1"][1, 0] = 1.0, -1.0
    P["W2"][0, 0], P["W2"][0, 1] = 1.0, 1.0
    P["b2"][1] = -3.0                     # a unit that stays off
    P["W2"][1, 0] = 1.0
    P["W3"][0, 0], P["W3"][1, 1] = 2.0, 5.0
    P["b3"][:] = [0.5, -1.0]
    X = np.zeros((3, Bu.NF))
    X[:, 0] = [3.0, -0.5, 1.0]            # standardised: 4, -3, 0
    out, _ = Bu.mlp_forward(th, X)
    # unit 0 of layer 2 = |x~0|, unit 1 = relu(relu(x~0) - 3)
    h = np.abs([4.0, -3.0, 0.0])
    u = np.maximum(np.maximum([4.0, -3.0, 0.0], 0) - 3.0, 0)
    assert np.allclose(out[:, 0], 2 * h + 0.5, rtol=0, atol=1e-15)
    assert np.allclose(out[:, 1], 5 * u - 1.0, rtol=0, atol=1e-15)
    # the output standardisation maps y~ to oshift + oscale y~
    P["oshift"][:] = [1.0, -2.0]
    P["oscale"][:] = [3.0, 0.5]
    out2, _ = Bu.mlp_forward(th, X)
    assert np.allclose(out2, [1.0, -2.0] + np.array([3.0, 0.5]) * out, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_matches_central_differences(seed):
    th, X, T = _net(seed)
    out, cache = Bu.mlp_forward(th, X)
    g = Bu.mlp_backward(th, cache, out, T)
    assert np.all(g[:Bu.NORM] == 0)
    rng = np.random.default_rng(100 + seed)
    idx = np.concatenate([rng.choice(np.arange(Bu.NORM, Bu.NPARAM), 300, replace=False),
                          np.arange(Bu.NPARAM - 130, Bu.NPARAM)])
    h = 1e-6
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        num = (Bu.mlp_loss(tp, Bu.mlp_forward(tp, X)[0], T) - Bu.mlp_loss(tm, Bu.mlp_forward(tm, X)[0], T)) / (2 * h)
        assert abs(num - g[k]) <= 1e-7 * max(1.0, abs(num)), (k, num, g[k])


def test_adam_closed_forms():
    g = np.random.default_rng(3)
    th0 = g.normal(0, 1, Bu.NPARAM)
    grad = g.normal(0, 1, Bu.NPARAM)
    m, v = np.zeros(Bu.NPARAM), np.zeros(Bu.NPARAM)
    th = Bu.adam_step(th0.copy(), grad, m, v, 1, lr=0.01, eps=0.0)
    # first step from zero moments: bias correction gives m^ = g, v^ = g^2
    s = slice(Bu.NORM, None)
    assert np.allclose(th[s], th0[s] - 0.01 * np.sign(grad[s]), rtol=0, atol=1e-15)
    assert np.array_equal(th[:Bu.NORM], th0[:Bu.NORM])
    # a constant gradient keeps m^ = g and v^ = g^2 at every step
    for t in range(2, 6):
        prev = th.copy()
        th = Bu.adam_step(th, grad, m, v, t, lr=0.01, eps=0.0)
        assert np.allclose(th[s] - prev[s], -0.01 * np.sign(grad[s]), rtol=0, atol=1e-13)


def test_normal_sf_matches_scipy():
    for z in [-6, -2.5, -1e-3, 0.0, 0.7, 1.96, 3.3, 8.0]:
        assert abs(Bu.normal_sf(z) - stats.norm.sf(z)) <= 1e-15 + 1e-13 * stats.norm.sf(z)


def test_budget_rule():
    zq = stats.norm.ppf(0.99)
    assert abs(zq - 2.3263478740408408) < 1e-12
    alpha = 0.05
    # p exactly alpha: no finite budget decides it -> the full budget
    z = stats.norm.isf(alpha)
    assert Bu.budgets(np.array([[0.0, 0.0]]), np.array([z]), alpha)[0] == 20000
    # far from alpha: the floor
    assert Bu.budgets(np.array([[0.0, 0.0]]), np.array([-3.0]), alpha)[0] == 200
    # in between: the formula, rounded up
    p = 0.03
    z = stats.norm.isf(p)
    want = math.ceil(zq * zq * p * (1 - p) / (p - alpha) ** 2)
    assert 200 < want < 20000
    assert Bu.budgets(np.array([[0.0, 0.0]]), np.array([z]), alpha)[0] == want
    # sigma scales z: mu = 1, sigma = e^0.5
    t = 1.0 + math.exp(0.5) * z
    assert Bu.budgets(np.array([[1.0, 0.5]]), np.array([t]), alpha)[0] == want
    # non-increasing as the predicted p moves away from alpha (either side)
    ps = np.linspace(0.001, 0.049, 30)
    b = [Bu.budgets(np.array([[0.0, 0.0]]), np.array([stats.norm.isf(q)]), alpha)[0] for q in ps]
    assert all(b[i] <= b[i + 1] for i in range(len(b) - 1))


def test_budget_band():
    """With a band [lo, hi]: inside -> the full budget; outside, the distance
    to the nearer edge replaces p - alpha."""
    zq = stats.norm.ppf(0.99)
    one = lambda p, lo, hi: Bu.budgets(np.array([[0.0, 0.0]]), np.array([stats.norm.isf(p)]), lo, hi)[0]
    for p in [0.02, 0.05, 0.0999]:
        assert one(p, 0.02, 0.10) == 20000
    p = 0.15
    assert one(p, 0.02, 0.10) == max(200, math.ceil(zq * zq * p * (1 - p) / (p - 0.10) ** 2))
    p = 0.012
    assert one(p, 0.02, 0.10) == max(200, math.ceil(zq * zq * p * (1 - p) / (p - 0.02) ** 2))
    # the point band is the plain rule
    assert one(0.03, 0.05, 0.05) == Bu.budgets(np.array([[0.0, 0.0]]), np.array([stats.norm.isf(0.03)]), 0.05)[0]


def test_features_against_aligned_clouds():
    """r(Z) and the angle term against the aligned rows themselves."""
    c = synth.small_pair_f64()
    a = O.align(c.X, c.Y)
    n, m, d = c.n, c.m, c.d
    f = Bu.features(n, m, d, a["r_x"], a["r_y"], a["vv"], a["t_obs"])
    assert f.shape == (12,)
    pooled = O.mrl(np.vstack([a["Xp"], c.Y]))
    assert abs(f[4] - pooled) <= 1e-12
    assert abs(f[5] - float(a["mu_x"] @ a["mu_y"])) <= 1e-12
    assert abs(f[8] - (f[7] - f[6])) <= 1e-12          # T_obs = f(r_Y) - f(r_X)
    assert abs(f[0] - math.log(n)) == 0 and abs(f[9] - n / (n + m)) <= 1e-15
    assert abs(f[10] - math.log(1 - a["r_x"] ** 2)) <= 1e-12


def test_null_moments():
    T = np.array([1.0, 2.0, 3.0, 6.0])
    mu, ls = Bu.null_moments(T)
    assert mu == 3.0 and abs(math.exp(ls) - math.sqrt(3.5)) < 1e-15


def test_training_reduces_loss():
    """Sanity of the pieces together: Adam on a small regression."""
    g = np.random.default_rng(9)
    X = g.normal(0, 1, (256, Bu.NF))
    T = np.stack([np.sin(X[:, 0]) + 0.5 * X[:, 1], 0.3 * X[:, 2] ** 2], 1)
    th = Bu.init_params(g)
    m, v = np.zeros(Bu.NPARAM), np.zeros(Bu.NPARAM)
    l0 = Bu.mlp_loss(th, Bu.mlp_forward(th, X)[0], T)
    for t in range(1, 301):
        out, cache = Bu.mlp_forward(th, X)
        Bu.adam_step(th, Bu.mlp_backward(th, cache, out, T), m, v, t, lr=3e-3)
    l1 = Bu.mlp_loss(th, Bu.mlp_forward(th, X)[0], T)
    assert l1 < 0.05 * l0
