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


def test_landing_probability_against_the_binomial():
    """The normal approximation of where the permutation p-value (1 + c) /
    (B + 1) lands, c ~ binomial(B, p): against scipy's exact binomial
    probabilities at large B (mean shifted by the +1, sd divided by B + 1)."""
    lo, hi = 0.02, 0.10
    for p, B in [(0.06, 8000), (0.11, 4096), (0.015, 8192), (0.3, 2000), (0.09, 16384)]:
        # c with lo <= (1 + c) / (B + 1) <= hi
        c_lo = math.ceil(lo * (B + 1) - 1)
        c_hi = math.floor(hi * (B + 1) - 1)
        exact = stats.binom.cdf(c_hi, B, p) - stats.binom.cdf(c_lo - 1, B, p)
        approx = Bu.land_prob(p, B, lo, hi)
        assert abs(approx - exact) <= 0.02, (p, B, approx, exact)
        # and the same normal probability through scipy's own normal
        mean, sd = (1 + B * p) / (B + 1), math.sqrt(B * p * (1 - p)) / (B + 1)
        assert abs(approx - (stats.norm.cdf((hi - mean) / sd) - stats.norm.cdf((lo - mean) / sd))) < 1e-12


def test_min_cost_budget_rule():
    """Inside the band: Bmax.  Far from it (p ~ 0 or p ~ 0.5): Bmin.  Just
    outside an edge the rule weighs more splits against the risk of a rerun:
    the budget it picks costs no more in expectation than Bmin or Bmax, and
    gets large (but below Bmax) at a moderate distance from the edge."""
    lo, hi, bmin, bmax = 0.02, 0.10, 64, 10000
    one = lambda p: Bu.budgets_min_cost(np.array([[0.0, 0.0]]), np.array([stats.norm.isf(p)]), lo, hi, bmin,
                                        bmax)[0]
    assert one(0.05) == bmax and one(0.0201) == bmax and one(0.0999) == bmax
    assert one(1e-9) == bmin and one(0.5) == bmin and one(0.9) == bmin
    cost = lambda p, B: B + bmax * Bu.land_prob(p, B, lo, hi) if B < bmax else bmax
    for p in [0.003, 0.012, 0.016, 0.105, 0.11, 0.12, 0.14, 0.2]:
        B = one(p)
        assert B == bmax or (B >= bmin and (B & (B - 1)) == 0 or B % bmin == 0)
        assert cost(p, B) <= cost(p, bmin) + 1e-9 and cost(p, B) <= bmax
    assert bmin < one(0.12) < bmax
    # the cost of a budget at p = 0.12 in numbers: 1024 splits leave a 2%
    # chance of landing in the band, 64 splits a 36% chance
    assert abs(Bu.land_prob(0.12, 1024, lo, hi) - stats.norm.cdf((0.10 - (1 + 1024 * 0.12) / 1025)
                                                               / (math.sqrt(1024 * 0.12 * 0.88) / 1025))) < 1e-3


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
