"""The rejection-rate experiment's shape on the GPU: 500 synthetic pairs,
B = 5,000 splits each, alpha = 0.05, a null and an alternative population, the
test without (naive) and with the Householder alignment.

Parity first (a few pairs of each population, both alignment modes, against
the FP64 oracle), then the statistical shape the paper reports: the aligned
test holds its level under a same-breadth null whose mean directions differ,
the naive test does not, and the aligned test still detects the breadth
difference of the alternative population.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_08048_amd import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_2605_08048_amd import rejection  # noqa: E402

ALPHA, NPAIRS, B = 0.05, 500, 5000
BAND = 3.0 * math.sqrt(ALPHA * (1.0 - ALPHA) / NPAIRS)


@pytest.fixture(scope="module")
def cells():
    out = {}
    for pop in ("null", "alt"):
        print(f"rejection population {pop}: {NPAIRS} pairs, B={B}", flush=True)
        b = synth.rejection_batch(pop, npairs=NPAIRS, B=B)
        out[pop] = (b, rejection.run_population(b, alpha=ALPHA))
    print({p: {k: out[p][1][k]["rate"] for k in ("naive", "aligned")} for p in out}, flush=True)
    return out


def test_counts_match_oracle_in_both_alignment_modes(cells):
    for pop, (b, r) in cells.items():
        small = np.argsort(b.n + b.m)[:3]
        for name, align in (("naive", 0), ("aligned", 1)):
            res = r[name]["results"]
            assert r[name]["status_ok"], (pop, name)
            for p in small:
                pr = b.pair(int(p))
                o = O.perm_test(pr.X, pr.Y, pr.B, seed=b.seed, pair=pr.pair_index, align=align, want_T=True)
                tie = int(np.sum(np.abs(o["T"] - o["t_obs"]) <= 1e-6 * abs(o["t_obs"])))
                assert abs(res[p]["t_obs"] - o["t_obs"]) <= 1e-12 * max(1.0, abs(o["t_obs"])), (pop, name, p)
                assert abs(int(res[p]["count"]) - o["count"]) <= tie, (pop, name, p)
                assert res[p]["p"] == (1.0 + res[p]["count"]) / (B + 1.0)


def test_observed_statistic_does_not_depend_on_the_alignment(cells):
    """T_obs is f(r_Y) - f(r_X) of the unreflected clouds (the reflection keeps
    r(X)), so both calls report the same value bit for bit; only the
    permutation distribution changes."""
    for pop, (b, r) in cells.items():
        for f in ("t_obs", "r_x", "r_y"):
            assert np.array_equal(r["naive"]["results"][f], r["aligned"]["results"][f]), (pop, f)


def test_aligned_test_holds_its_level_and_the_naive_test_does_not(cells):
    naive, aligned = cells["null"][1]["naive"]["rate"], cells["null"][1]["aligned"]["rate"]
    assert abs(aligned - ALPHA) <= BAND, aligned
    assert naive > ALPHA + BAND, naive


def test_aligned_test_detects_the_breadth_difference(cells):
    null, alt = cells["null"][1]["aligned"]["rate"], cells["alt"][1]["aligned"]["rate"]
    assert alt > null + BAND, (null, alt)
