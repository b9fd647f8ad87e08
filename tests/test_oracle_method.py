"""Pins of the oracle's arithmetic against facts the paper and mathematics fix.

Sections of the paper: Sec. 3.1 (mean directions, Householder axis and
reflection, MRL, g_d, eq:tobs, eq:pvalue), Algorithm 1, and the appendix
"Proof Sketch" (pooled MRL after alignment).  Each check comes from outside
the oracle: closed forms, a library routine, brute-force enumeration or a
statistical property.
"""
from itertools import combinations
from math import comb

import numpy as np
import pytest
from scipy import special, stats

from oracle import oracle as O
from paper_2605_08048_amd import synth


def _pair(n, m, d, kx=3.0, ky=3.0, angle=40.0, seed=0):
    g = np.random.default_rng(seed)
    mu = synth.random_unit(g, d)
    mv = synth.direction_at_angle(g, mu, angle)
    X = synth.unit_rows(kx * mu + g.standard_normal((n, d)) / np.sqrt(d))
    Y = synth.unit_rows(ky * mv + g.standard_normal((m, d)) / np.sqrt(d))
    return X, Y


# ---------------------------------------------------------------- Householder

def _H(v):
    return np.eye(v.size) - 2.0 * np.outer(v, v) / (v @ v)


def test_means_and_directions_match_numpy():
    X, Y = _pair(30, 45, 12)
    a = O.align(X, Y)
    assert abs(a["r_x"] - np.linalg.norm(X.mean(0))) < 1e-14
    assert abs(a["r_y"] - np.linalg.norm(Y.mean(0))) < 1e-14
    assert np.allclose(a["mu_x"], X.mean(0) / np.linalg.norm(X.mean(0)), atol=1e-14)
    assert np.allclose(a["v"], a["mu_x"] - a["mu_y"], atol=0)


@pytest.mark.parametrize("d", [3, 64, 768])
def test_householder_closed_forms(d):
    X, Y = _pair(40, 50, d, angle=70.0, seed=d)
    a = O.align(X, Y)
    H = _H(a["v"])
    # H mu_x = mu_y and H^T H = H^2 = I (Sec. 3.1)
    assert np.linalg.norm(H @ a["mu_x"] - a["mu_y"]) < 1e-12
    assert np.abs(H @ H - np.eye(d)).max() < 1e-12
    # the aligned rows are exactly H x_i, norms kept
    assert np.abs(a["Xp"] - X @ H.T).max() < 1e-12
    assert np.abs(np.linalg.norm(a["Xp"], axis=1) - 1).max() < 1e-12
    # reflecting twice gives X back
    assert np.abs(a["Xp"] @ H.T - X).max() < 1e-12
    # dispersion unchanged: r(X') = r(X)
    assert abs(np.linalg.norm(a["Xp"].mean(0)) - a["r_x"]) < 1e-12
    # the mean direction of X' is mu_y
    mx = a["Xp"].mean(0)
    assert np.linalg.norm(mx / np.linalg.norm(mx) - a["mu_y"]) < 1e-12


def test_householder_hand_example_swaps_axes():
    # mu_x = e1, mu_y = e2: H swaps coordinates 1 and 2 and keeps the rest.
    d = 5
    X = np.zeros((4, d))
    X[:, 0] = 1.0
    X[1] = [0.6, 0.8, 0, 0, 0]
    X[3] = [0.6, -0.8, 0, 0, 0]
    Y = np.zeros((2, d))
    Y[:, 1] = 1.0
    Y[1] = [0.0, 0.6, 0.8, 0, 0]
    Y[0] = [0.0, 0.6, -0.8, 0, 0]
    a = O.align(X, Y)
    assert np.allclose(a["mu_x"], [1, 0, 0, 0, 0]) and np.allclose(a["mu_y"], [0, 1, 0, 0, 0])
    assert np.allclose(a["Xp"], X[:, [1, 0, 2, 3, 4]], atol=1e-15)


def test_pooled_mrl_after_alignment_proof_sketch():
    # Appendix "Proof Sketch": with R = H the pooled MRL reaches its bound
    # (n r_X + m r_Y) / (n + m), and the total sum is (n r_X + m r_Y) mu_y.
    X, Y = _pair(70, 30, 20, angle=100.0, seed=3)
    a = O.align(X, Y)
    Z = np.vstack([a["Xp"], Y])
    n, m = X.shape[0], Y.shape[0]
    bound = (n * a["r_x"] + m * a["r_y"]) / (n + m)
    assert abs(np.linalg.norm(Z.mean(0)) - bound) < 1e-12
    assert np.linalg.norm(Z.sum(0) - (n * a["r_x"] + m * a["r_y"]) * a["mu_y"]) < 1e-11
    # any other orthogonal map does no better (random rotations)
    g = np.random.default_rng(0)
    for _ in range(5):
        Q, _ = np.linalg.qr(g.standard_normal((20, 20)))
        assert np.linalg.norm(np.vstack([X @ Q.T, Y]).mean(0)) <= bound + 1e-12


def test_identity_when_directions_coincide_or_alignment_off():
    X, Y = _pair(20, 25, 8)
    a = O.align(X, X.copy())
    assert a["h_identity"] == 1 and np.array_equal(a["Xp"], X)
    b = O.align(X, Y, align=0)
    assert b["h_identity"] == 1 and np.array_equal(b["Xp"], X)


# ---------------------------------------------------------------- MRL, g_d, T

def test_mrl_closed_forms():
    v = synth.random_unit(np.random.default_rng(1), 9)
    assert abs(O.mrl(np.tile(v, (7, 1))) - 1.0) < 1e-15
    assert O.mrl(np.vstack([v, -v, v, -v])) < 1e-15
    k = 7
    ang = 2 * np.pi * np.arange(k) / k
    assert O.mrl(np.stack([np.cos(ang), np.sin(ang)], 1)) < 1e-15
    A = synth.unit_rows(np.random.default_rng(2).standard_normal((50, 6)))
    assert abs(O.mrl(A) - np.linalg.norm(A.mean(0))) < 1e-15


@pytest.mark.parametrize("d,tol", [(3, 0.025), (16, 0.01), (64, 3e-3), (768, 3e-4)])
def test_banerjee_g_inverts_vmf_mean_resultant(d, tol):
    # The vMF mean resultant length is A_d(kappa) = I_{d/2}(kappa) / I_{d/2-1}(kappa);
    # g_d(r) estimates the kappa with A_d(kappa) = r (Banerjee et al. 2005).
    for r in [0.1, 0.3, 0.6, 0.9, 0.97]:
        kappa = np.exp(O.log_g(r, d))
        A = special.ive(d / 2, kappa) / special.ive(d / 2 - 1, kappa)
        assert abs(A - r) / r < tol, (d, r, kappa, A)


def test_g_monotone_and_identity_variant():
    rs = np.linspace(0.01, 0.99, 200)
    f = np.array([O.log_g(r, 768) for r in rs])
    assert np.all(np.diff(f) > 0)
    assert O.log_g(0.37, 768, O.GD_IDENTITY) == np.log(0.37)


def test_tobs_sign_broader_x_is_positive():
    # v = 1 / g_d(r): the broader cloud has the smaller r and the larger v,
    # so "u (= X) broader than k (= Y)" means T_obs > 0.
    X, Y = _pair(200, 200, 32, kx=1.2, ky=3.0, seed=4)
    a = O.align(X, Y)
    assert a["r_x"] < a["r_y"] and a["t_obs"] > 0


def test_tobs_identical_groups_is_exactly_zero_and_antisymmetric():
    X, Y = _pair(25, 31, 10, seed=5)
    assert O.perm_test(X, X.copy(), B=20)["t_obs"] == 0.0
    a, b = O.align(X, Y), O.align(Y, X)
    assert a["t_obs"] == -b["t_obs"]
    assert O.align(X, Y, align=0)["t_obs"] == a["t_obs"]


def test_observed_split_reproduces_tobs():
    # Group 1 = the first n pooled rows (X') is the observed labelling; its
    # permuted statistic must equal T_obs.
    X, Y = _pair(13, 21, 7, kx=2.0, ky=3.0, seed=6)
    a = O.align(X, Y)
    Z = np.vstack([a["Xp"], Y])
    sel = np.zeros(34, bool)
    sel[:13] = True
    T, r1, r2 = O.split_stat(Z, 13, 21, O.bool_to_mask(sel)[0])
    assert abs(T - a["t_obs"]) < 1e-12
    assert abs(r1 - a["r_x"]) < 1e-13 and abs(r2 - a["r_y"]) < 1e-13


# ---------------------------------------------------------------- p-values

def _brute_exact_p(X, Y, align=1):
    a = O.align(X, Y, align=align)
    Z = np.vstack([a["Xp"], Y])
    n, m = X.shape[0], Y.shape[0]
    d = X.shape[1]
    f = lambda r: np.log(r * (d - r * r) / (1 - r * r))
    Ts = []
    for c in combinations(range(n + m), n):
        s = np.zeros(n + m, bool)
        s[list(c)] = True
        Ts.append(f(np.linalg.norm(Z[~s].mean(0))) - f(np.linalg.norm(Z[s].mean(0))))
    Ts = np.array(Ts)
    return Ts, a["t_obs"], a["tau"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exhaustive_70_splits_match_brute_force_and_scipy(seed):
    X, Y = _pair(4, 4, 5, kx=1.5, ky=2.5, angle=60.0, seed=10 + seed)
    ex = O.exhaustive(X, Y, want_T=True)
    assert ex["total"] == comb(8, 4) == 70
    Ts, tobs, tau = _brute_exact_p(X, Y)
    assert np.abs(np.sort(ex["T"]) - np.sort(Ts)).max() < 1e-12
    assert ex["count"] == int(np.sum(Ts >= tobs - tau))
    assert ex["count"] >= 1                         # the observed split counts
    # scipy's exact permutation test over the same 70 splits (rows looked up by index)
    a = O.align(X, Y)
    Z = np.vstack([a["Xp"], Y])
    d = 5
    f = lambda r: np.log(r * (d - r * r) / (1 - r * r))
    stat = lambda i, j: f(np.linalg.norm(Z[np.asarray(j, int)].mean(0))) - f(np.linalg.norm(Z[np.asarray(i, int)].mean(0)))
    res = stats.permutation_test((np.arange(4), np.arange(4, 8)), stat, permutation_type="independent",
                                 n_resamples=np.inf, alternative="greater", vectorized=False)
    assert abs(res.pvalue - ex["p"]) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_exhaustive_two_sided_p_matches_scipy_when_null_is_symmetric(seed):
    """Two-sided rule (|T_b| >= |T_obs|; the paper reports two-sided values
    without a definition).  With n = m every split's complement is also a
    split and gives -T_b, so the exact null distribution is symmetric and the
    rule must equal scipy's two-sided exact p (twice the smaller one-sided
    p).  A dropped absolute value or a wrong sign of the threshold fails."""
    X, Y = _pair(4, 4, 5, kx=1.5 + 0.5 * seed, ky=2.5, angle=60.0, seed=30 + seed)
    ex = O.exhaustive(X, Y, alternative=O.ALT_TWO_SIDED)
    a = O.align(X, Y)
    Z = np.vstack([a["Xp"], Y])
    d = 5
    f = lambda r: np.log(r * (d - r * r) / (1 - r * r))
    stat = lambda i, j: f(np.linalg.norm(Z[np.asarray(j, int)].mean(0))) - f(np.linalg.norm(Z[np.asarray(i, int)].mean(0)))
    res = stats.permutation_test((np.arange(4), np.arange(4, 8)), stat, permutation_type="independent",
                                 n_resamples=np.inf, alternative="two-sided", vectorized=False)
    assert abs(res.pvalue - ex["p"]) < 1e-12, (res.pvalue, ex["p"])
    # the swapped problem reflects with the same H and has T_obs -> -T_obs
    sw = O.exhaustive(Y, X, alternative=O.ALT_TWO_SIDED)
    assert sw["count"] == ex["count"]


def test_monte_carlo_p_converges_to_exact_p():
    X, Y = _pair(5, 5, 6, kx=2.0, ky=2.5, angle=50.0, seed=21)
    ex = O.exhaustive(X, Y)
    B = 20000
    mc = O.perm_test(X, Y, B=B, seed=9)
    assert abs(mc["p"] - (1 + mc["count"]) / (B + 1)) < 1e-15
    pe = ex["p"]
    assert abs(mc["p"] - pe) <= 4 * np.sqrt(pe * (1 - pe) / B) + 1.0 / B


def test_p_floor_and_plus_one():
    # X much broader than Y: no split beats the observed one in a modest B.
    X, Y = _pair(60, 60, 16, kx=0.6, ky=4.0, seed=22)
    r = O.perm_test(X, Y, B=199)
    assert r["count"] == 0 and r["p"] == 1.0 / 200


def test_perm_offset_splitting_is_additive():
    X, Y = _pair(30, 41, 9, kx=2.0, ky=2.2, seed=23)
    full = O.perm_test(X, Y, B=300, seed=4, want_T=True)
    a = O.perm_test(X, Y, B=120, seed=4, want_T=True)
    b = O.perm_test(X, Y, B=180, seed=4, perm_offset=120, want_T=True)
    assert full["count"] == a["count"] + b["count"]
    assert np.array_equal(full["T"], np.concatenate([a["T"], b["T"]]))


def test_explicit_masks_reproduce_philox_run_and_reject_bad_masks():
    X, Y = _pair(17, 12, 5, seed=24)
    r = O.perm_test(X, Y, B=50, seed=2, want_masks=True, want_T=True)
    again = O.perm_test(X, Y, B=50, masks=r["masks"], want_T=True)
    assert again["count"] == r["count"] and np.array_equal(again["T"], r["T"])
    bad = r["masks"].copy()
    bad[3, 0] ^= 1
    assert O.perm_test(X, Y, B=50, masks=bad)["status"] == O.ERR_MASK


def test_two_sided_counts_both_tails():
    X, Y = _pair(40, 40, 8, kx=1.0, ky=3.0, seed=25)
    g = O.perm_test(X, Y, B=400, seed=1, want_T=True)
    t = O.perm_test(X, Y, B=400, seed=1, alternative=O.ALT_TWO_SIDED)
    assert t["count"] == int(np.sum(np.abs(g["T"]) >= abs(g["t_obs"]) - g["tau"]))


def test_rows_that_are_not_unit_vectors_are_flagged():
    """Eq. 2 normalises every embedding; a row off by more than 1e-4 in norm
    (or NaN) is reported, one off by 5e-5 is not."""
    X, Y = _pair(30, 20, 8, seed=26)
    assert O.align(X, Y)["status"] == O.OK
    for scale, status in [(1 + 2e-4, O.ERR_NOT_UNIT), (1 - 2e-4, O.ERR_NOT_UNIT), (1 + 5e-5, O.OK)]:
        Xs = X.copy()
        Xs[7] *= scale
        assert O.align(Xs, Y)["status"] == status
        Ys = Y.copy()
        Ys[19] *= scale
        assert O.perm_test(X, Ys, B=10)["status"] == status
    Xn = X.copy()
    Xn[0, 3] = np.nan
    assert O.align(Xn, Y)["status"] in (O.ERR_NOT_UNIT, O.ERR_DEGENERATE)


def test_degenerate_single_direction_is_flagged():
    v = synth.random_unit(np.random.default_rng(3), 4)
    X = np.tile(v, (5, 1))
    Y = synth.unit_rows(np.random.default_rng(4).standard_normal((6, 4)))
    assert O.align(X, Y)["status"] == O.ERR_DEGENERATE


# ---------------------------------------------------------------- calibration

def _null_rates(R, n, d, B, align):
    """Same-breadth null (equal kappa), means 40 degrees apart, isotropic noise."""
    rej = 0
    for k in range(R):
        g = np.random.default_rng([77, k])
        mu = synth.random_unit(g, d)
        mv = synth.direction_at_angle(g, mu, 40.0)
        X = synth.unit_rows(2.0 * mu + g.standard_normal((n, d)) / np.sqrt(d) * 1.5)
        Y = synth.unit_rows(2.0 * mv + g.standard_normal((n, d)) / np.sqrt(d) * 1.5)
        rej += O.perm_test(X, Y, B=B, seed=k, align=align)["p"] <= 0.05
    return rej / R


def test_type_one_error_near_alpha_for_same_breadth_null():
    R = 600
    rate = _null_rates(R, 40, 16, 199, align=1)
    band = 3 * np.sqrt(0.05 * 0.95 / R)
    assert abs(rate - 0.05) <= band, rate


def test_naive_test_rejects_too_often_when_directions_differ():
    """The failure mode the alignment removes (Sec. 1, Fig. 1): with equal
    breadth and equal group sizes, pooling two clouds whose mean directions
    differ lowers every permuted r, which narrows the naive null of T, so the
    naive test rejects well above alpha; the aligned test on the same pairs
    stays at alpha.  (With very unequal n and m the share of X rows in a
    permuted group varies to first order and widens the naive null instead.)"""
    R, d, B = 300, 32, 199
    fac = synth.lowrank_factor(d)
    rej = {0: 0, 1: 0}
    for k in range(R):
        g = np.random.default_rng([78, k])
        n = int(g.integers(60, 160))
        X, Y = synth._lowrank_pair(60, k, n, n, d, 3.0, 3.0, angle=60.0, factor=fac)
        for a in (0, 1):
            rej[a] += O.perm_test(X, Y, B=B, seed=k, align=a)["p"] <= 0.05
    band = 3 * np.sqrt(0.05 * 0.95 / R)
    assert abs(rej[1] / R - 0.05) <= band, rej
    assert rej[0] / R > 0.05 + band, rej


def test_power_when_x_is_broader():
    rej = 0
    for k in range(60):
        X, Y = _pair(80, 80, 16, kx=1.4, ky=2.6, seed=1000 + k)
        rej += O.perm_test(X, Y, B=199, seed=k)["p"] <= 0.05
    assert rej >= 55
