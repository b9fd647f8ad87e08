"""Learned permutation-budget allocator: control flow over the C ABI.

The permutation test of the paper spends the same number of random splits
on every pair.  Here a small network (12 -> 64 -> 64 -> 2, FP32; the
kernels are in ``csrc/budget.hip``) estimates each pair's permutation null
distribution of T from the quantities of the alignment stage, and that
estimate decides how many splits the pair gets:

1. every pair is tested with ``b_first`` splits (``b_min`` without the
   network); this also yields the alignment quantities the network reads,
   which need no splits at all, so with the network ``b_first`` can be small;
2. the network's (mean, log sd) and the pair's T_obs give a normal
   approximation p^; the pair gets B_p splits (b_max when p^ lies in the
   fallback band [p_lo, p_hi]; otherwise the budget from b_min, 2 b_min, ...,
   b_max with the least expected splits, counting a rerun at b_max when its
   p lands in the band, or with rule "zq" enough splits to put ``zq``
   standard errors between p^ and the band); the extra B_p - b_first splits
   continue the same
   counter-based stream (``perm_offset = b_first``), so the counts simply
   add;
3. pairs whose permutation p lands in [p_lo, p_hi] are tested again with the
   full ``b_max`` splits from split 0 (the full-budget result itself).

Without the network every pair gets the same b_min, which has to be large
enough for any pair; with it, pairs whose p^ is far from the band get a
smaller floor and pairs near the band get enough splits that their p does not
land in the band by Monte Carlo noise alone (each such landing costs b_max).

The decision is always the exact permutation p-value of eq:pvalue.  This
module only marshals arguments and moves host-side arrays (budgets, the
pair subsets of the later stages) between ABI calls; every computation runs
in the library's kernels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import hbt

ZQ_99 = 2.3263478740408408   # standard normal 0.99 quantile


def init_theta(rng: np.random.Generator) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, identity
    standardisations; the draws for W1, W2, W3 come from ``rng`` in that order."""
    th = np.zeros(hbt.MLP_PARAMS, dtype=np.float64)
    F, H = hbt.MLP_FEATURES, 64
    th[F:2 * F] = 1.0
    th[2 * F + 2:2 * F + 4] = 1.0
    o = hbt.MLP_TRAINABLE_OFFSET
    for rows, cols in ((H, F), (H, H), (2, H)):
        lim = math.sqrt(6.0 / cols)
        th[o:o + rows * cols] = rng.uniform(-lim, lim, rows * cols)
        o += rows * cols + rows
    return th


@dataclass
class Allocator:
    theta: "object"                       # float32 device tensor, MLP_PARAMS
    m: "object" = None
    v: "object" = None
    step: int = 0
    history: list = field(default_factory=list)

    @classmethod
    def create(cls, device, seed=0, theta=None):
        import torch
        th = init_theta(np.random.default_rng(seed)) if theta is None else np.asarray(theta)
        t = torch.tensor(th, dtype=torch.float32, device=device)
        return cls(t, torch.zeros_like(t), torch.zeros_like(t))

    def fit(self, features, targets, steps=500, lr=3e-3, normalise=True):
        """Full-batch Adam on the mean half squared error of the standardised
        targets; returns the loss of every step."""
        import torch
        if normalise and self.step == 0:
            hbt.feature_norm(features, self.theta)
            hbt.target_norm(targets, self.theta)
        grad = None
        hist = torch.empty(steps, dtype=torch.float64, device=self.theta.device)
        for i in range(steps):  # step i writes its loss (before its update) into hist[i]
            grad, _ = hbt.mlp_grad(features, targets, self.theta, grad, hist[i:i + 1])
            self.step += 1
            hbt.mlp_adam(self.theta, grad, self.m, self.v, self.step, lr)
        out = hist.cpu().numpy().tolist()
        self.history += out
        return out

    def predict(self, features):
        return hbt.mlp_forward(features, self.theta)


def adaptive_perm_test(Z_all, row_offset, n, m, allocator=None, *, d=None, seed=0, precision="bf16x2",
                       gd="banerjee", p_lo=0.02, p_hi=0.10, b_min=200, b_max=20000, zq=ZQ_99,
                       b_first=None, rule="cost"):
    """The three-stage test above; ``allocator=None`` skips stage 2 (every
    pair keeps b_min unless stage 3 applies).  ``b_first`` (default b_min,
    at most b_min) is the first stage's splits.  ``rule``: "cost" (the
    budget with the least expected splits, hbt_budgets_min_cost) or "zq"
    (zq standard errors from the band, hbt_budgets).  Returns per-pair numpy
    arrays and the number of splits each stage evaluated."""
    P = len(n)
    d = Z_all.shape[1] if d is None else d
    b_first = b_min if b_first is None else int(b_first)
    if not 1 <= b_first <= b_min:
        raise ValueError("b_first must lie in [1, b_min]")
    if allocator is None:
        b_first = b_min
    off = np.asarray(row_offset[:P], dtype=np.int64)
    nn, mm = np.asarray(n, dtype=np.int64), np.asarray(m, dtype=np.int64)
    ids = np.arange(P, dtype=np.uint32)
    kw = dict(seed=seed, precision=precision, gd=gd)
    # stage 1
    r1 = hbt.perm_test_batched(Z_all, off, nn, mm, np.full(P, b_first), pair_index=ids, sync=False, **kw)
    res = hbt.results_to_numpy(r1)
    count = res["count"].astype(np.int64)
    B = np.full(P, b_first, dtype=np.int64)
    splits = {"stage1": int(P * b_first), "stage2": 0, "stage3": 0}
    # stage 2
    if allocator is not None:
        feat = hbt.budget_features(r1, d, gd)
        out = allocator.predict(feat)
        if rule == "cost":
            Bp = hbt.budgets_min_cost(out, r1, p_lo, p_hi, b_min, b_max).cpu().numpy()
        elif rule == "zq":
            Bp = hbt.budgets(out, r1, p_lo, p_hi, b_min, b_max, zq).cpu().numpy()
        else:
            raise ValueError(f"unknown budget rule {rule!r}")
        more = np.nonzero(Bp > b_first)[0]
        if more.size:
            r2 = hbt.perm_test_batched(Z_all, off[more], nn[more], mm[more], Bp[more] - b_first,
                                       pair_index=ids[more], perm_offset=b_first, **kw)
            count[more] += r2["count"]
            B[more] = Bp[more]
            splits["stage2"] = int(np.sum(Bp[more] - b_first))
    p = (1.0 + count) / (B + 1.0)
    B0 = B.copy()
    # stage 3
    redo = np.nonzero((p >= p_lo) & (p <= p_hi) & (B < b_max))[0]
    if redo.size:
        r3 = hbt.perm_test_batched(Z_all, off[redo], nn[redo], mm[redo], np.full(redo.size, b_max),
                                   pair_index=ids[redo], **kw)
        count[redo] = r3["count"]
        B[redo] = b_max
        p[redo] = r3["p"]
        splits["stage3"] = int(redo.size * b_max)
    splits["total"] = splits["stage1"] + splits["stage2"] + splits["stage3"]
    splits["pairs_at_b_max_before_stage3"] = int(np.sum(B0 >= b_max)) if allocator is not None else 0
    return dict(p=p, count=count, B=B, t_obs=res["t_obs"], splits=splits, reran=redo)
