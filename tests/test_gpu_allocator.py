"""GPU: the allocator kernels (through the C ABI) against the FP64 reference
oracle/budget.py, then what a trained network gains over a fixed budget.

Bars: features and targets to FP32 rounding of the FP64 values; forward and
gradient within FP32 accumulation bounds (n u times the magnitudes, n the
longest dot product); Adam to FP32 rounding; budgets identical (both sides
take the integer decision in FP64 from the same FP32 network outputs).
"""
import math

import numpy as np
import pytest

from oracle import budget as Bu
from oracle import oracle as O
from paper_2605_08048_amd import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_2605_08048_amd import allocator as A  # noqa: E402
from paper_2605_08048_amd import hbt  # noqa: E402

DEV = "cuda:0"
U32 = 2.0 ** -24


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _theta(seed):
    """A random network with non-zero biases and a standardisation, rounded to
    FP32 (the FP64 reference then starts from exactly the same numbers)."""
    g = np.random.default_rng(seed)
    th = A.init_theta(g)
    P = Bu.unpack(th)
    P["shift"][:] = g.normal(0, 1, Bu.NF)
    P["scale"][:] = g.uniform(0.5, 2.0, Bu.NF)
    P["b1"][:] = g.normal(0, 0.3, Bu.H1)
    P["b2"][:] = g.normal(0, 0.3, Bu.H2)
    P["b3"][:] = g.normal(0, 0.3, Bu.NO)
    P["oshift"][:] = g.normal(0, 1, Bu.NO)
    P["oscale"][:] = g.uniform(0.2, 3.0, Bu.NO)
    return th.astype(np.float32).astype(np.float64)


def _small_batch(P=9, d=96, seed=3):
    g = np.random.default_rng(seed)
    pairs = []
    for p in range(P):
        n, m = int(g.integers(4, 300)), int(g.integers(4, 300))
        mu = synth.random_unit(g, d)
        mv = synth.direction_at_angle(g, mu, float(g.uniform(5, 60)))
        X = synth.unit_rows(g.uniform(1.5, 3) * mu + g.standard_normal((n, d)) / math.sqrt(d))
        Y = synth.unit_rows(g.uniform(1.5, 3) * mv + g.standard_normal((m, d)) / math.sqrt(d))
        pairs.append(synth.Pair(X.astype(np.float32), Y.astype(np.float32), B=500, pair_index=p))
    return pairs, synth.pack_batch(pairs, d)


def test_features_and_targets_match_reference():
    pairs, b = _small_batch()
    res = hbt.perm_test_batched(_dev(b.Z), b.row_offset, b.n, b.m, b.B, seed=5, precision="f32", sync=False)
    feat = hbt.budget_features(res, b.d).cpu().numpy().astype(np.float64)
    tg = hbt.null_targets(res).cpu().numpy().astype(np.float64)
    rec = hbt.results_to_numpy(res)
    for p, pr in enumerate(pairs):
        a = O.align(pr.X, pr.Y)
        want = Bu.features(pr.X.shape[0], pr.Y.shape[0], b.d, a["r_x"], a["r_y"], a["vv"], a["t_obs"])
        # FP32 rounding of values computed in FP64 from inputs equal to 1e-12
        assert np.allclose(feat[p], want, rtol=2 * U32, atol=1e-9), (p, feat[p] - want)
        assert tg[p, 0] == np.float32(rec["t_mean"][p])
        assert abs(tg[p, 1] - math.log(rec["t_sd"][p])) <= U32 * abs(math.log(rec["t_sd"][p])) * 1.01


def test_feature_norm_matches_numpy():
    g = np.random.default_rng(1)
    X = (g.normal(0, 1, (1000, 12)) * g.uniform(0.1, 10, 12) + g.normal(0, 5, 12)).astype(np.float32)
    X[:, 7] = 2.5  # a constant feature keeps scale 1
    th = torch.zeros(hbt.MLP_PARAMS, dtype=torch.float32, device=DEV)
    hbt.feature_norm(_dev(X), th)
    t = th.cpu().numpy()
    X64 = X.astype(np.float64)
    mean, sd = X64.mean(0), X64.std(0)
    assert np.allclose(t[:12], mean, rtol=U32 * 2, atol=1e-7)
    ok = sd > 0
    assert np.allclose(t[12:24][ok], 1.0 / sd[ok], rtol=4 * U32, atol=0)
    assert t[12 + 7] == 1.0 and np.all(t[24:] == 0)


def test_target_norm_matches_numpy():
    g = np.random.default_rng(5)
    T = np.stack([g.normal(0.01, 0.02, 500), g.normal(-3, 0.5, 500)], 1).astype(np.float32)
    th = torch.zeros(hbt.MLP_PARAMS, dtype=torch.float32, device=DEV)
    hbt.target_norm(_dev(T), th)
    t = th.cpu().numpy()
    T64 = T.astype(np.float64)
    assert np.allclose(t[24:26], T64.mean(0), rtol=2 * U32, atol=1e-9)
    assert np.allclose(t[26:28], T64.std(0), rtol=4 * U32, atol=0)
    assert np.all(t[:24] == 0) and np.all(t[28:] == 0)


def _magnitude(th, X):
    """Forward pass of |network| on |inputs|: bounds the size of every partial sum."""
    P = Bu.unpack(np.abs(th))
    Xs = np.abs((X - Bu.unpack(th)["shift"]) * P["scale"])
    Z1 = Xs @ P["W1"].T + P["b1"]
    Z2 = Z1 @ P["W2"].T + P["b2"]
    return P["oshift"] + P["oscale"] * (Z2 @ P["W3"].T + P["b3"])


@pytest.mark.parametrize("seed", [0, 1])
def test_forward_matches_reference(seed):
    th = _theta(seed)
    X = np.random.default_rng(10 + seed).normal(0, 2, (777, 12)).astype(np.float32).astype(np.float64)
    out = hbt.mlp_forward(_dev(X), _dev(th)).cpu().numpy()
    want, _ = Bu.mlp_forward(th, X)
    tol = 3 * 80 * U32 * _magnitude(th, X)
    assert np.all(np.abs(out - want) <= tol), np.max(np.abs(out - want) / tol)


@pytest.mark.parametrize("rows", [1, 333, 1000])
def test_gradient_matches_reference(rows):
    th = _theta(rows)
    g = np.random.default_rng(rows)
    X = g.normal(0, 2, (rows, 12)).astype(np.float32).astype(np.float64)
    T = g.normal(0, 1, (rows, 2)).astype(np.float32).astype(np.float64)
    grad, loss = hbt.mlp_grad(_dev(X), _dev(T), _dev(th))
    grad, loss = grad.cpu().numpy().astype(np.float64), float(loss.item())
    out, cache = Bu.mlp_forward(th, X)
    want = Bu.mlp_backward(th, cache, out, T)
    assert abs(loss - Bu.mlp_loss(th, out, T)) <= 1e-5 * Bu.mlp_loss(th, out, T)
    assert np.all(grad[:Bu.NORM] == 0)
    # FP32 per-row error signals (relative error ~ 200 u), FP64 sums over rows
    scale = np.abs(want).max()
    assert np.allclose(grad, want, rtol=400 * 4 * U32, atol=1e-4 * scale), np.max(np.abs(grad - want))


def test_adam_matches_reference():
    g = np.random.default_rng(4)
    th = g.normal(0, 1, hbt.MLP_PARAMS).astype(np.float32)
    grad = g.normal(0, 1e-2, hbt.MLP_PARAMS).astype(np.float32)
    m = g.normal(0, 1e-2, hbt.MLP_PARAMS).astype(np.float32)
    v = g.uniform(0, 1e-4, hbt.MLP_PARAMS).astype(np.float32)
    t_th, t_m, t_v = _dev(th), _dev(m), _dev(v)
    hbt.mlp_adam(t_th, _dev(grad), t_m, t_v, 7, lr=1e-3)
    th64, m64, v64 = th.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    # the kernel's hyper-parameters are float32: the reference uses the same values
    f = lambda x: float(np.float32(x))
    Bu.adam_step(th64, grad.astype(np.float64), m64, v64, 7, lr=f(1e-3), b1=f(0.9), b2=f(0.999), eps=f(1e-8))
    got = t_th.cpu().numpy()
    assert np.array_equal(got[:24], th[:24])
    # about eight FP32 roundings in the update, one in the final subtraction
    delta = np.abs(th64 - th.astype(np.float64))
    assert np.all(np.abs(got - th64) <= U32 * (np.abs(th64) + 8 * delta) + 1e-12)
    assert np.all(np.abs(t_m.cpu().numpy() - m64) <= 4 * U32 * (0.9 * np.abs(m) + 0.1 * np.abs(grad)))
    assert np.allclose(t_v.cpu().numpy(), v64, rtol=4 * U32, atol=1e-15)


def test_budgets_match_reference():
    pairs, b = _small_batch(P=40, d=32, seed=8)
    res = hbt.perm_test_batched(_dev(b.Z), b.row_offset, b.n, b.m, b.B, seed=5, precision="f32", sync=False)
    t_obs = hbt.results_to_numpy(res)["t_obs"]
    g = np.random.default_rng(2)
    # outputs that put p^ on both sides of and inside the band
    sd = np.exp(g.uniform(-5, -1, 40))
    z = g.uniform(-4, 4, 40)
    out = np.stack([t_obs - z * sd, np.log(sd)], 1).astype(np.float32)
    for lo, hi, bmin, bmax in [(0.02, 0.10, 200, 20000), (0.05, 0.05, 100, 5000)]:
        got = hbt.budgets(_dev(out), res, lo, hi, bmin, bmax).cpu().numpy()
        want = Bu.budgets(out.astype(np.float64), t_obs, lo, hi, bmin, bmax)
        assert np.array_equal(got, want), (lo, hi, got - want)
        assert got.min() >= bmin and got.max() <= bmax
        got = hbt.budgets_min_cost(_dev(out), res, lo, hi, bmin, bmax).cpu().numpy()
        want = Bu.budgets_min_cost(out.astype(np.float64), t_obs, lo, hi, bmin, bmax)
        assert np.array_equal(got, want), (lo, hi, got - want)
        assert got.min() >= bmin and got.max() <= bmax


def test_training_follows_reference():
    """Full-batch Adam on the GPU against the FP64 reference from the same start."""
    g = np.random.default_rng(9)
    X = g.normal(0, 1, (256, 12)).astype(np.float32).astype(np.float64)
    T = np.stack([np.sin(X[:, 0]) + 0.5 * X[:, 1], 0.3 * X[:, 2] ** 2], 1).astype(np.float32).astype(np.float64)
    th0 = A.init_theta(np.random.default_rng(0)).astype(np.float32).astype(np.float64)
    al = A.Allocator.create(DEV, theta=th0)
    gpu = al.fit(_dev(X), _dev(T), steps=60, lr=3e-3, normalise=False)
    th, m, v = th0.copy(), np.zeros_like(th0), np.zeros_like(th0)
    ref = []
    for t in range(1, 61):
        out, cache = Bu.mlp_forward(th, X)
        ref.append(Bu.mlp_loss(th, out, T))
        Bu.adam_step(th, Bu.mlp_backward(th, cache, out, T), m, v, t, lr=3e-3)
    assert abs(gpu[0] - ref[0]) <= 1e-5 * ref[0]
    assert abs(gpu[-1] - ref[-1]) <= 2e-2 * ref[-1], (gpu[-1], ref[-1])
    assert gpu[-1] < 0.5 * gpu[0]


def test_trained_allocator_gain_over_fixed_budget_and_no_network():
    """Train the network on null statistics the method itself produces, then
    compare on held-out pairs: splits spent and decisions at alpha = 0.05
    against every pair at the full budget (the paper's fixed B), and against
    the same procedure without the network (b_min plus the fallback band).
    The adaptive runs use a seed independent of both reference runs.  The
    network must spend fewer splits than the procedure without it, with as
    many decision changes as two full-budget runs with different seeds."""
    from paper_2605_08048_amd import budget_run
    print("allocator gain: 1500 training and 1000 held-out pairs of the budget workload at d=256", flush=True)
    r = budget_run.run(train=1500, test=1000, d=256, b_train=2000, b_max=10000, chunk=1250, steps=800,
                       log=lambda s: print(s, flush=True))
    print({k: r[k] for k in ("fixed", "net", "base", "net_stage3", "base_stage3", "dis_full", "dis_net",
                             "dis_base", "rejections", "mse_net", "mse_constant")}, flush=True)
    # the network learned the null spread (log sd) far better than a constant
    assert r["mse_net"][1] < 0.25 * r["mse_constant"][1]
    # decisions as the full budget, up to Monte Carlo noise
    assert r["dis_net"] <= r["dis_full"] + 3
    # fewer splits than without the network, and a fraction of the fixed budget
    assert r["net"] < r["base"], (r["net"], r["base"])
    assert r["net"] <= 0.4 * r["fixed"]
