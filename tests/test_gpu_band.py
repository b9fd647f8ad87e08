"""GPU: raw reduced-precision statistics against the recheck band, and counts
on inputs whose rows repeat.

The FP64 recheck only re-evaluates splits whose T_b lies within the band of
the threshold (hbt_recheck_band), so every raw T_b of a reduced precision must
lie within that band of the FP64 value, including the accumulation error of
the product (which the CPU emulation of the stored rows leaves out).  The
cases are the hard ones: a group of 2, r near 1, diffuse clouds (r ~ 0.03),
rows repeated up to 500 times, d up to 8192, and both statistic routes.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_08048_amd import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_2605_08048_amd import hbt  # noqa: E402

DEV = "cuda:0"


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def _cloud(g, n, d, kappa, mu, rep):
    """n unit rows around mu: n // rep distinct rows, each repeated rep times,
    in random order."""
    k = max(1, n // rep)
    base = synth.unit_rows(kappa * mu + g.standard_normal((k, d)) / math.sqrt(d))
    idx = np.concatenate([np.arange(k)] * (n // k + 1))[:n]
    g.shuffle(idx)
    return base[idx].astype(np.float32)


def _pair(n, m, d, kx, ky, rep=1, seed=0, angle=40.0):
    g = np.random.default_rng([13, seed, n, m, d, rep])
    mu = synth.random_unit(g, d)
    mv = synth.direction_at_angle(g, mu, angle)
    return _cloud(g, n, d, kx, mu, rep), _cloud(g, m, d, ky, mv, rep)


RAW_CASES = [
    # n, m, d, kappa_x, kappa_y, repeats
    (2, 300, 64, 8.0, 8.0, 1), (2, 61, 1024, 30.0, 30.0, 1), (3, 500, 16, 4.0, 6.0, 1),
    (400, 350, 768, 2.0, 2.2, 1), (1000, 2, 256, 12.0, 12.0, 1), (37, 41, 1024, 40.0, 45.0, 1),
    (1000, 1000, 768, 2.0, 2.4, 100), (1000, 1000, 768, 2.0, 2.4, 500),
    (1000, 1000, 768, 0.03, 0.03, 1), (3000, 2000, 1024, 0.02, 0.02, 1),
    (1000, 1000, 768, 0.03, 0.03, 500), (2, 2000, 768, 0.05, 0.05, 1),
]


@pytest.mark.parametrize("prec,route", [("f32", 0), ("bf16x2", 0), ("i8x3", 0), ("bf16e4m3", 0),
                                        ("f32", 1), ("bf16x2", 1), ("f64", 1)])
def test_raw_errors_stay_inside_the_recheck_band(prec, route):
    """Without the recheck, |T_b - T_b(FP64)| <= band / 2 for every split."""
    worst = 0.0
    cases = RAW_CASES + ([(101, 157, 8192, 2.0, 2.1, 1), (300, 200, 8192, 0.05, 0.05, 1),
                          (400, 400, 8192, 2.0, 2.2, 100)] if route == 1 else [])
    for n, m, d, kx, ky, rep in cases:
        print(f"raw band {prec} route {route}: n={n} m={m} d={d} rep={rep}", flush=True)
        X, Y = _pair(n, m, d, kx, ky, rep, seed=n * 7 + d)
        B = 300
        r = hbt.perm_test(_dev(X), _dev(Y), B, seed=11, precision=prec, recheck=False, want_T="f64",
                          stat_route=route)
        at = O.perm_stats_at(X, Y, np.arange(B), seed=11)
        eps = hbt.recheck_band(prec, n, m, d, at["r1"], at["r2"], stat_route=route)
        ratio = np.abs(r["T"] - at["T"]) / eps
        worst = max(worst, float(ratio.max()))
        assert ratio.max() <= 0.5, (prec, route, n, m, d, rep, float(ratio.max()))
    print(f"{prec} route {route}: worst |T - T64| / band = {worst:.3g}")


# null pairs (equal concentration), so that T_obs sits inside the permutation
# distribution and many splits fall near it
REPEAT_CASES = [(1000, 1000, 768, 2.2, 10), (1000, 1000, 768, 2.2, 100), (1000, 1000, 768, 2.2, 500),
                (1500, 900, 1024, 0.03, 300), (700, 2100, 768, 0.03, 1)]


@pytest.mark.parametrize("prec", ["bf16x2", "i8x3", "bf16e4m3"])
def test_repeated_rows_counts_match_oracle(prec):
    """Clouds built from few distinct rows, and diffuse clouds: the counts of
    the single-pair call and of the batched call equal the oracle's."""
    pairs = []
    for k, (n, m, d, kappa, rep) in enumerate(REPEAT_CASES):
        X, Y = _pair(n, m, d, kappa, kappa, rep, seed=50 + k, angle=30.0)
        pairs.append((X, Y, d))
    B = 2000
    for k, (X, Y, d) in enumerate(pairs):
        print(f"repeated rows {prec} single pair {REPEAT_CASES[k]}", flush=True)
        r = hbt.perm_test(_dev(X), _dev(Y), B, seed=3, pair_index=k, precision=prec)
        o = O.perm_test(X, Y, B, seed=3, pair=k, want_T=True)
        tie = int(np.sum(np.abs(o["T"] - o["t_obs"]) <= 1e-6 * abs(o["t_obs"])))
        print(f"  count {r['count']} (oracle {o['count']}), rechecked {r['n_recheck']}", flush=True)
        assert r["status"] == 0
        assert abs(r["count"] - o["count"]) <= tie, (prec, k, r["count"], o["count"])
    # the d = 768 pairs in one batched call
    sel = [k for k, c in enumerate(REPEAT_CASES) if c[2] == 768]
    bt = synth.pack_batch([synth.Pair(pairs[k][0], pairs[k][1], B=B, pair_index=k) for k in sel], 768)
    print(f"repeated rows {prec} batched, {len(sel)} pairs", flush=True)
    res = hbt.perm_test_batched(_dev(bt.Z), bt.row_offset, bt.n, bt.m, bt.B, seed=3,
                                pair_index=np.array(sel, dtype=np.uint32), precision=prec)
    for j, k in enumerate(sel):
        o = O.perm_test(pairs[k][0], pairs[k][1], B, seed=3, pair=k, want_T=True)
        tie = int(np.sum(np.abs(o["T"] - o["t_obs"]) <= 1e-6 * abs(o["t_obs"])))
        assert res[j]["status"] == 0
        assert abs(res[j]["count"] - o["count"]) <= tie, (prec, k, res[j]["count"], o["count"])
        print(f"  pair {k}: count {res[j]['count']} (oracle {o['count']}), rechecked {res[j]['n_recheck']}",
              flush=True)


def test_repeated_rows_counts_match_oracle_lazy():
    """The lazy precision (batched call) on the same clouds: its first
    pass decides from the hi plane alone, whose rounding errors add up
    coherently over repeated rows; counts must equal the oracle's and the
    split-BF16 call's, pair by pair."""
    B = 2000
    for d in (768, 1024):
        sel = [k for k, c in enumerate(REPEAT_CASES) if c[2] == d]
        pairs = []
        for k in sel:
            n, m, _, kappa, rep = REPEAT_CASES[k]
            X, Y = _pair(n, m, d, kappa, kappa, rep, seed=50 + k, angle=30.0)
            pairs.append(synth.Pair(X, Y, B=B, pair_index=k))
        bt = synth.pack_batch(pairs, d)
        print(f"repeated rows lazy batched d={d}, {len(sel)} pairs", flush=True)
        Z = _dev(bt.Z)
        ids = np.array(sel, dtype=np.uint32)
        lz = hbt.perm_test_batched(Z, bt.row_offset, bt.n, bt.m, bt.B, seed=3, pair_index=ids, precision="bf16lazy")
        sb = hbt.perm_test_batched(Z, bt.row_offset, bt.n, bt.m, bt.B, seed=3, pair_index=ids, precision="bf16x2")
        for j, pr in enumerate(pairs):
            o = O.perm_test(pr.X, pr.Y, B, seed=3, pair=pr.pair_index, want_T=True)
            tie = int(np.sum(np.abs(o["T"] - o["t_obs"]) <= 1e-6 * abs(o["t_obs"])))
            assert lz[j]["status"] == 0
            assert abs(lz[j]["count"] - o["count"]) <= tie, (d, j, lz[j]["count"], o["count"])
            assert lz[j]["count"] == sb[j]["count"] and lz[j]["n_recheck"] == sb[j]["n_recheck"], (d, j)
            print(f"  pair {pr.pair_index}: count {lz[j]['count']} (oracle {o['count']}), "
                  f"rechecked {lz[j]['n_recheck']}", flush=True)
