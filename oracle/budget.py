"""FP64 reference of the learned permutation-budget allocator.

TEST INFRASTRUCTURE ONLY: used by ``tests/`` (and nothing in the product
library imports it).  Plain numpy, FP64, no batching tricks beyond a matrix
product per layer, so each step can be checked against its definition.

The allocator predicts, from cheap per-pair quantities of the alignment stage,
the location and spread of a pair's permutation null distribution of T, and
turns the implied normal-approximation p-value into a number of permutations
large enough to decide p against alpha.  The exact permutation p-value of the
method (Sec. 3.1, eq:pvalue) stays the decision; pairs whose p lands near
alpha are completed to the full budget.  The paper itself uses a fixed number
of permutations per pair; this part is an addition built on its statistic.

Pieces:
* ``features``   12 numbers per pair (Sec. 3.1 quantities: group sizes, mean
  resultant lengths, the pooled MRL after alignment, the angle between the
  mean directions, log g_d, the observed statistic);
* ``mlp_*``      a 12 -> 64 -> 64 -> 2 ReLU network with fixed input and
  output standardisations, its squared-error loss (on standardised
  targets), and backpropagation;
* ``adam_step``  Adam (Kingma & Ba 2015, Algorithm 1, bias-corrected);
* ``budgets``    B = clamp(ceil(zq^2 p(1-p) / (p - e)^2), Bmin, Bmax) with
  p = 1 - Phi((T_obs - mu) / sigma) and e the nearer edge of the fallback
  band [lo, hi] (Bmax inside the band; lo = hi = alpha is the plain rule);
* ``budgets_min_cost``  the B (Bmin doubling, or Bmax) with the least
  expected splits B + Bmax * P(p lands in the band after B splits).
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O

NF, H1, H2, NO = 12, 64, 64, 2
NORM = 2 * NF + 2 * NO                # input shift/scale, output shift/scale (not trained)
SHAPES = [("shift", (NF,)), ("scale", (NF,)), ("oshift", (NO,)), ("oscale", (NO,)),
          ("W1", (H1, NF)), ("b1", (H1,)),
          ("W2", (H2, H1)), ("b2", (H2,)),
          ("W3", (NO, H2)), ("b3", (NO,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)   # 5150


def unpack(theta):
    """Views of the flat parameter vector, in the order of SHAPES (row-major)."""
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def init_params(rng, shift=None, scale=None):
    """He-uniform weights, zero biases; shifts default to 0, scales to 1."""
    theta = np.zeros(NPARAM)
    P = unpack(theta)
    P["shift"][:] = 0.0 if shift is None else shift
    P["scale"][:] = 1.0 if scale is None else scale
    P["oscale"][:] = 1.0
    for w, fan in (("W1", NF), ("W2", H1), ("W3", H2)):
        lim = math.sqrt(6.0 / fan)
        P[w][:] = rng.uniform(-lim, lim, P[w].shape)
    return theta


# ------------------------------------------------------------------ features

def features(n, m, d, r_x, r_y, vv, t_obs, gd=O.GD_BANERJEE):
    """The 12 inputs of one pair.

    r(Z) is the MRL of the pooled aligned set; after the Householder map both
    means point along mu_y, so ||sum z|| = n r_X + m r_Y (appendix, proof of
    the alignment optimum).  cos(angle) between the unit mean directions is
    1 - |mu_x - mu_y|^2 / 2 = 1 - vv / 2.
    """
    N = n + m
    fx, fy = O.log_g(r_x, d, gd), O.log_g(r_y, d, gd)
    return np.array([math.log(n), math.log(m), r_x, r_y, (n * r_x + m * r_y) / N, 1.0 - vv / 2.0,
                     fx, fy, t_obs, n / N, math.log1p(-r_x * r_x), math.log1p(-r_y * r_y)])


# ------------------------------------------------------------------ network

def mlp_forward(theta, X):
    """X (rows x 12) -> (out (rows x 2), cache); out = oshift + oscale * y~,
    y~ the last layer's value."""
    P = unpack(theta)
    Xs = (X - P["shift"]) * P["scale"]
    A1 = Xs @ P["W1"].T + P["b1"]
    Z1 = np.maximum(A1, 0.0)
    A2 = Z1 @ P["W2"].T + P["b2"]
    Z2 = np.maximum(A2, 0.0)
    Yt = Z2 @ P["W3"].T + P["b3"]
    return P["oshift"] + P["oscale"] * Yt, (Xs, A1, Z1, A2, Z2)


def mlp_loss(theta, out, target):
    """Mean over rows of half the squared error of the standardised outputs,
    (out - target) / oscale, summed over the 2 outputs."""
    e = (out - target) / unpack(theta)["oscale"]
    return 0.5 * float(np.sum(e ** 2)) / out.shape[0]


def mlp_backward(theta, cache, out, target):
    """Gradient of mlp_loss with respect to theta (zero for the standardisations)."""
    P = unpack(theta)
    Xs, A1, Z1, A2, Z2 = cache
    R = out.shape[0]
    g = np.zeros_like(theta)
    G = unpack(g)
    dO = (out - target) / P["oscale"] / R   # d loss / d y~
    G["W3"][:] = dO.T @ Z2
    G["b3"][:] = dO.sum(0)
    dA2 = (dO @ P["W3"]) * (A2 > 0)
    G["W2"][:] = dA2.T @ Z1
    G["b2"][:] = dA2.sum(0)
    dA1 = (dA2 @ P["W2"]) * (A1 > 0)
    G["W1"][:] = dA1.T @ Xs
    G["b1"][:] = dA1.sum(0)
    return g


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, first=NORM):
    """One Adam update (step number t >= 1) of theta[first:], in place; returns theta."""
    s = slice(first, None)
    m[s] = b1 * m[s] + (1.0 - b1) * grad[s]
    v[s] = b2 * v[s] + (1.0 - b2) * grad[s] ** 2
    mh = m[s] / (1.0 - b1 ** t)
    vh = v[s] / (1.0 - b2 ** t)
    theta[s] -= lr * mh / (np.sqrt(vh) + eps)
    return theta


# ------------------------------------------------------------------ budget

def normal_sf(z):
    """1 - Phi(z) through the complementary error function."""
    return 0.5 * math.erfc(z / math.sqrt(2.0))


def budgets(out, t_obs, lo=0.05, hi=None, bmin=200, bmax=20000, zq=2.3263478740408408):
    """Permutations per pair from the network outputs (mu, log sigma)."""
    hi = lo if hi is None else hi
    B = np.empty(out.shape[0], dtype=np.int64)
    for i in range(out.shape[0]):
        mu, ls = float(out[i, 0]), float(out[i, 1])
        p = normal_sf((float(t_obs[i]) - mu) / math.exp(ls))
        if lo <= p <= hi:
            B[i] = bmax
            continue
        e = lo if p < lo else hi
        need = zq * zq * p * (1.0 - p) / (p - e) ** 2
        B[i] = bmax if need >= bmax else max(bmin, int(math.ceil(need)))
    return B


def land_prob(p, B, lo, hi):
    """Probability that the permutation p-value (1 + count) / (B + 1) of a
    pair with p-value p lands in [lo, hi], the count binomial(B, p) taken as
    normal (mean B p, variance B p (1 - p))."""
    mean = (1.0 + B * p) / (B + 1.0)
    sd = math.sqrt(B * p * (1.0 - p)) / (B + 1.0)
    if not sd > 0.0:
        return 1.0 if lo <= mean <= hi else 0.0
    return normal_sf((lo - mean) / sd) - normal_sf((hi - mean) / sd)


def budgets_min_cost(out, t_obs, lo, hi, bmin, bmax):
    """Permutations per pair minimising the expected splits: Bmax inside the
    band; otherwise the B in {Bmin 2^k < Bmax} u {Bmax} with the least
    B + Bmax * land_prob(p, B) (the smaller B on ties)."""
    B = np.empty(out.shape[0], dtype=np.int64)
    for i in range(out.shape[0]):
        mu, ls = float(out[i, 0]), float(out[i, 1])
        p = normal_sf((float(t_obs[i]) - mu) / math.exp(ls))
        if lo <= p <= hi:
            B[i] = bmax
            continue
        cands = []
        c = bmin
        while c < bmax:
            cands.append(c)
            c *= 2
        best, bestB = float(bmax), bmax
        for c in cands:
            cost = c + bmax * land_prob(p, c, lo, hi)
            if cost < best:
                best, bestB = cost, c
        B[i] = bestB
    return B


def null_moments(T):
    """Targets of one pair from its permuted statistics: (mean, log sd)."""
    T = np.asarray(T, dtype=np.float64)
    mu = T.mean()
    return np.array([mu, 0.5 * math.log(np.mean((T - mu) ** 2))])
