"""Rejection rates of the naive and the aligned test over a population of pairs.

The shape of the paper's rejection-rate experiment (the table of rejection
rates under a null and an alternative condition, Sec. 4 experiments across
corpora): many pairs, one fixed split budget per pair, alpha = 0.05, the
permutation test run once without the Householder alignment (the baseline)
and once with it.  A rate under the null estimates the Type-I error, a rate
under the alternative the power.

Every statistic, split and count comes from one batched library call per
(population, alignment) cell; this module only uploads the synthetic clouds
of ``synth.rejection_batch``, makes those calls and counts p <= alpha on the
host.

    python -m paper_2605_08048_amd.rejection [--pairs 500] [--B 5000]
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from . import hbt, synth


def run_population(batch, *, alpha=0.05, precision="bf16x2", alternative="greater", device="cuda:0"):
    """Both tests on one population: per-pair results of the naive and the
    aligned call, and their rejection rates at ``alpha``."""
    import torch
    Z = torch.as_tensor(batch.Z, device=device)
    out = {}
    for name, align in (("naive", False), ("aligned", True)):
        res = hbt.perm_test_batched(Z, batch.row_offset, batch.n, batch.m, batch.B, seed=batch.seed,
                                    pair_index=batch.pair_index, precision=precision,
                                    alternative=alternative, align=align)
        out[name] = dict(results=res, rate=float(np.mean(res["p"] <= alpha)),
                         status_ok=bool(np.all(res["status"] == 0)))
    del Z
    return out


def table(npairs=500, B=5000, d=768, alpha=0.05, precision="bf16x2", alternative="greater", device="cuda:0"):
    """Rejection rates for the null and the alternative population."""
    rows = {}
    for pop in ("null", "alt"):
        b = synth.rejection_batch(pop, npairs=npairs, d=d, B=B)
        r = run_population(b, alpha=alpha, precision=precision, alternative=alternative, device=device)
        rows[pop] = {k: r[k]["rate"] for k in ("naive", "aligned")}
    band = 3.0 * math.sqrt(alpha * (1.0 - alpha) / npairs)
    return dict(pairs=npairs, B=B, d=d, alpha=alpha, precision=precision, alternative=alternative,
                band_3sd=band, rates=rows)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--pairs", type=int, default=500)
    ap.add_argument("--B", type=int, default=5000)
    ap.add_argument("--alpha", type=float, default=0.05)
    ap.add_argument("--precision", default="bf16x2", choices=sorted(hbt.PRECISION))
    ap.add_argument("--alternative", default="greater", choices=["greater", "two-sided"])
    a = ap.parse_args(argv)
    t = table(a.pairs, a.B, alpha=a.alpha, precision=a.precision, alternative=a.alternative)
    print(f"{'population':<12}{'naive':>8}{'aligned':>9}")
    for pop, label in (("null", "null"), ("alt", "alternative")):
        r = t["rates"][pop]
        print(f"{label:<12}{r['naive']:>8.3f}{r['aligned']:>9.3f}")
    print(json.dumps(t))


if __name__ == "__main__":
    main()
