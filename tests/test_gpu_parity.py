"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars (per result, against FP64):
  * random splits and their masks: bit-exact;
  * Householder: r, T_obs in FP64 to 1e-12; aligned rows in the input dtype;
  * permuted statistics T_b: |T_gpu - T_64| <= tol * (|f(r1)| + |f(r2)|) with
    tol = 1e-10 (F64), 1e-5 (F32), 1e-4 (split BF16, int8 digit planes);
  * exceedance counts: equal, except for splits with |T_64 - T_obs| <=
    1e-6 |T_obs| (none of which occur in these cases, so counts are equal);
  * p = (1 + count) / (B + 1) exactly.
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
TOL = {"f64": 1e-10, "f32": 1e-5, "bf16x2": 1e-4, "i8x3": 1e-4, "bf16e4m3": 1e-4,
       # the lazy precision: its T_b outside the hi plane's
       # band carry the hi plane's error; its null moments are held to this
       "bf16lazy": 5e-4}


def _dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _logg(r, d):
    return np.log(r * (d - r * r) / (1 - r * r))


def _scale(X, Y, ora_at):
    d = X.shape[1]
    return np.abs(_logg(ora_at["r1"], d)) + np.abs(_logg(ora_at["r2"], d))


def _tie_band(T64, tobs):
    return int(np.sum(np.abs(T64 - tobs) <= 1e-6 * abs(tobs)))


def _pair(n, m, d, kx=2.0, ky=2.4, angle=40.0, seed=0, f64=False):
    g = np.random.default_rng([5, seed])
    mu = synth.random_unit(g, d)
    mv = synth.direction_at_angle(g, mu, angle)
    X = synth.unit_rows(kx * mu + g.standard_normal((n, d)) / math.sqrt(d))
    Y = synth.unit_rows(ky * mv + g.standard_normal((m, d)) / math.sqrt(d))
    if not f64:
        X, Y = X.astype(np.float32), Y.astype(np.float32)
    return X, Y


# --------------------------------------------------------------------- align

@pytest.mark.parametrize("f64", [False, True])
def test_align_matches_oracle(f64):
    print(f"align f64={f64}", flush=True)
    X, Y = _pair(300, 257, 100, seed=1, f64=f64)
    r = hbt.align(_dev(X), _dev(Y))
    o = O.align(X, Y)
    assert r["status"] == 0 and r["h_identity"] == 0
    assert abs(r["r_x"] - o["r_x"]) < 1e-12 and abs(r["r_y"] - o["r_y"]) < 1e-12
    assert abs(r["t_obs"] - o["t_obs"]) < 1e-12 * max(1, abs(o["t_obs"]))
    assert np.abs(r["v"].cpu().numpy() - o["v"]).max() < 1e-13
    Xp = r["X_out"].cpu().numpy().astype(np.float64)
    ulp = 1e-15 if f64 else 2e-7
    assert np.abs(Xp - o["Xp"]).max() <= ulp * 4
    # The Householder checks on the GPU's own output: H built from the
    # returned v sends the input's mean direction to Y's (1e-12), applying H
    # to the returned rows gives back X (H^2 = I), and the returned rows keep
    # r(X' ) = r(X) (H is orthogonal).  FP64 input: to 1e-12; FP32 rows: to
    # their rounding.
    v = r["v"].cpu().numpy()
    H = np.eye(X.shape[1]) - 2.0 * np.outer(v, v) / (v @ v)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    mux = X64.mean(0) / np.linalg.norm(X64.mean(0))
    muy = Y64.mean(0) / np.linalg.norm(Y64.mean(0))
    assert np.linalg.norm(H @ mux - muy) <= 1e-12
    tol = 1e-12 if f64 else 1e-6
    assert np.abs(Xp @ H.T - X64).max() <= tol
    assert abs(np.linalg.norm(Xp.mean(0)) - np.linalg.norm(X64.mean(0))) <= tol
    assert abs(np.linalg.norm(Xp.mean(0)) - r["r_x"]) <= tol


def test_align_in_place_and_identity():
    X, Y = _pair(64, 70, 33, seed=2)
    Xd = _dev(X)
    o = O.align(X, Y)
    r = hbt.align(Xd, _dev(Y), out=Xd)
    assert np.abs(Xd.cpu().numpy() - o["Xp"]).max() < 1e-6
    r0 = hbt.align(_dev(X), _dev(Y), align=False)
    assert r0["h_identity"] == 1 and np.array_equal(r0["X_out"].cpu().numpy(), X)
    same = hbt.align(_dev(X), _dev(X))
    assert same["h_identity"] == 1 and same["t_obs"] == 0.0


def test_non_unit_rows_are_reported():
    """Rows must be unit vectors (Sec. 3.1, Eq. 2); a row whose norm is off by
    more than 1e-4 gives the pair the status NOT_UNIT, as in the oracle, on
    every path that sums the columns (16-byte loads, the scalar path for FP64
    input or d not a multiple of 4, the batched call); 5e-5 passes."""
    for d, f64 in [(100, False), (100, True), (50, False)]:
        X, Y = _pair(300, 257, d, seed=3, f64=f64)
        cases = {"x": (X.copy(), Y, True), "y": (X, Y.copy(), True), "ok": (X.copy(), Y, False)}
        cases["x"][0][17] *= 1.001
        cases["y"][1][200] *= 0.999
        cases["ok"][0][5] *= 1.0 + 5e-5
        for name, (Xc, Yc, bad) in cases.items():
            want = hbt.ERR_NOT_UNIT if bad else 0
            print(f"non-unit rows d={d} f64={f64} {name}", flush=True)
            assert O.perm_test(Xc, Yc, 5)["status"] == (O.ERR_NOT_UNIT if bad else O.OK)
            assert hbt.align(_dev(Xc), _dev(Yc))["status"] == want, (d, f64, name)
            for prec in ["f32", "bf16x2"]:
                assert hbt.perm_test(_dev(Xc), _dev(Yc), 20, precision=prec)["status"] == want, (d, f64, name, prec)
    X, Y = _pair(300, 257, 96, seed=4)
    pairs = [synth.Pair(X, Y, B=50, pair_index=p) for p in range(3)]
    Xb = X.copy()
    Xb[250] *= 1.01
    Yb = Y.copy()
    Yb[3] *= 0.99
    pairs[0] = synth.Pair(Xb, Y, B=50, pair_index=0)
    pairs[2] = synth.Pair(X, Yb, B=50, pair_index=2)
    bt = synth.pack_batch(pairs, 96)
    for prec in ["bf16x2", "i8x3", "f32"]:
        res = hbt.perm_test_batched(_dev(bt.Z), bt.row_offset, bt.n, bt.m, bt.B, precision=prec)
        assert list(res["status"]) == [hbt.ERR_NOT_UNIT, 0, hbt.ERR_NOT_UNIT], prec


# --------------------------------------------------------------------- splits

# (4000, 7), (16380, 7): group 1 ends in the top key byte, next to the padding
# of the last Philox block; N > 16384 regenerates keys instead of holding them
@pytest.mark.parametrize("n,m", [(4, 4), (2, 61), (50, 60), (777, 3), (1000, 1048), (2000, 1500), (5000, 4999),
                                 (4000, 7), (16380, 7), (9000, 8000), (40000, 25536)])
def test_masks_bit_exact(n, m):
    print(f"masks n={n} m={m}", flush=True)
    N = n + m
    d = 8
    X, Y = _pair(n, m, d, seed=3)
    B = 64
    for seed, pair, off in [(0, 0, 0), (123456789012345, 77, 4000000000)]:
        r = hbt.perm_test(_dev(X), _dev(Y), B, seed=seed, pair_index=pair, perm_offset=off,
                          precision="f32", want_masks=True)
        got = r["masks"]
        assert got.shape == (B, (N + 31) // 32)
        want = np.stack([O.split_mask(seed, pair, off + b, N, n) for b in range(B)])
        assert np.array_equal(got, want)
        assert r["status"] == 0


# --------------------------------------------------------------------- full test, small shapes

CASES = [
    # n, m, d, B, precision, f64-input
    (50, 60, 64, 999, "f64", True),     # the FP64 correctness configuration
    (37, 150, 100, 700, "f64", False),
    (37, 150, 100, 700, "f32", False),  # ragged d (pad to 128) and ragged N
    (150, 37, 100, 700, "f32", False),  # n > m: the product runs on group 2
    (37, 150, 100, 700, "bf16x2", False),
    (150, 37, 100, 700, "bf16x2", False),
    (300, 450, 768, 600, "bf16x2", False),
    (300, 450, 768, 600, "f32", False),
    (40, 70, 37, 300, "f32", False),    # d % 4 != 0: the scalar-load alignment kernels
    (70, 40, 37, 300, "bf16x2", False),
    (50, 60, 64, 999, "i8x3", True),    # int8 digit planes: FP64 input, exact integer sums
    (37, 150, 100, 700, "i8x3", False),
    (150, 37, 100, 700, "i8x3", False),
    (300, 450, 768, 600, "i8x3", False),
    (70, 40, 37, 300, "i8x3", False),
    (2, 5000, 1024, 300, "i8x3", False),  # the smallest group, widest supported d in one slot set
    (101, 157, 1030, 300, "bf16x2", False),  # d_pad 1088: past the 16-byte-load alignment kernels
    (101, 157, 8192, 200, "f32", False),     # the largest d the library accepts
    (101, 157, 8192, 200, "bf16x2", False),
    (157, 101, 8192, 200, "i8x3", False),
    (50, 60, 64, 999, "bf16e4m3", True),      # BF16 hi + e4m3 lo: FP64 input (row-at-a-time alignment)
    (37, 150, 100, 700, "bf16e4m3", False),
    (150, 37, 100, 700, "bf16e4m3", False),
    (300, 450, 768, 600, "bf16e4m3", False),
    (70, 40, 37, 300, "bf16e4m3", False),
    (101, 157, 1030, 300, "bf16e4m3", False),
    (101, 157, 8192, 200, "bf16e4m3", False),
    (9000, 8000, 64, 100, "bf16e4m3", False),  # many 32-row groups and lo units per pair
    (9000, 8000, 64, 100, "bf16x2", False),
    (50, 60, 64, 999, "bf16lazy", True),       # lazy split BF16: FP64 input
    (150, 37, 100, 700, "bf16lazy", False),
    (300, 450, 768, 600, "bf16lazy", False),
    (70, 40, 37, 300, "bf16lazy", False),
    (101, 157, 1030, 300, "bf16lazy", False),
    (101, 157, 8192, 200, "bf16lazy", False),
    (9000, 8000, 64, 100, "bf16lazy", False),
]


@pytest.mark.parametrize("n,m,d,B,prec,f64", CASES)
def test_perm_test_matches_oracle(n, m, d, B, prec, f64):
    print(f"perm_test n={n} m={m} d={d} B={B} {prec} f64={f64}", flush=True)
    X, Y = _pair(n, m, d, kx=2.0, ky=2.1, seed=n + m + d, f64=f64)
    r = hbt.perm_test(_dev(X), _dev(Y), B, seed=7, precision=prec, want_T=True)
    o = O.perm_test(X, Y, B, seed=7, want_T=True)
    at = O.perm_stats_at(X, Y, np.arange(B), seed=7)
    assert r["status"] == 0
    assert abs(r["t_obs"] - o["t_obs"]) <= 1e-12 * max(1.0, abs(o["t_obs"]))
    err = np.abs(r["T"].astype(np.float64) - o["T"]) / _scale(X, Y, at)
    # T_out is rounded to float32 on output: allow its half-ulp on top of the bar
    assert err.max() <= TOL[prec] + 1.2e-7, err.max()
    band = _tie_band(o["T"], o["t_obs"])
    assert abs(r["count"] - o["count"]) <= band
    assert r["B"] == B and r["p"] == (1 + r["count"]) / (B + 1)
    _check_extras(r, o, n, m, _scale(X, Y, at), prec)


def _check_extras(r, o, n, m, scale, prec):
    """mu_cos, group sizes and the null moments of T_b against the oracle.  The
    mean moves by at most the per-split bar; the SD by at most twice it."""
    assert r["n"] == n and r["m"] == m
    assert abs(r["mu_cos"] - (1 - o["vv"] / 2)) <= 1e-12
    tol = (TOL[prec] + 1.2e-7) * np.max(scale)
    assert abs(r["t_mean"] - o["T"].mean()) <= tol, (r["t_mean"], o["T"].mean())
    assert abs(r["t_sd"] - o["T"].std()) <= 2 * tol, (r["t_sd"], o["T"].std())


def test_identical_groups_give_zero_and_count_all_ties():
    X, _ = _pair(40, 40, 32, seed=9)
    r = hbt.perm_test(_dev(X), _dev(X.copy()), 500, precision="f32")
    o = O.perm_test(X, X.copy(), 500)
    assert r["t_obs"] == 0.0 and r["h_identity"] == 1
    assert r["count"] == o["count"]


def test_exhaustive_70_splits_with_explicit_masks():
    X, Y = _pair(4, 4, 16, kx=1.5, ky=2.5, angle=60.0, seed=11, f64=True)
    from itertools import combinations
    sel = np.zeros((70, 8), bool)
    for k, c in enumerate(combinations(range(8), 4)):
        sel[k, list(c)] = True
    masks = O.bool_to_mask(sel)
    ex = O.exhaustive(X, Y)
    for prec in ["f64", "f32", "bf16x2", "i8x3", "bf16e4m3"]:
        r = hbt.perm_test(_dev(X), _dev(Y), 70, precision=prec, masks=masks)
        assert r["status"] == 0
        assert r["count"] == ex["count"]
        assert r["count"] / 70 == ex["p"]


def test_bad_explicit_mask_is_reported():
    X, Y = _pair(10, 12, 8, seed=12)
    masks = np.stack([O.split_mask(0, 0, b, 22, 10) for b in range(5)])
    masks[2, 0] ^= 1
    r = hbt.perm_test(_dev(X), _dev(Y), 5, masks=masks)
    assert r["status"] == hbt.ERR_MASK


@pytest.mark.parametrize("prec", ["f32", "bf16x2", "i8x3", "bf16e4m3"])
def test_block_size_offsets_and_repeat_do_not_change_results(prec):
    X, Y = _pair(500, 700, 128, kx=2.0, ky=2.05, seed=13)
    Xd, Yd = _dev(X), _dev(Y)
    full = hbt.perm_test(Xd, Yd, 3000, seed=5, precision=prec, want_T=True)
    again = hbt.perm_test(Xd, Yd, 3000, seed=5, precision=prec, want_T=True)
    blocked = hbt.perm_test(Xd, Yd, 3000, seed=5, precision=prec, block_perms=700, want_T=True)
    a = hbt.perm_test(Xd, Yd, 1234, seed=5, precision=prec)
    b = hbt.perm_test(Xd, Yd, 3000 - 1234, seed=5, perm_offset=1234, precision=prec)
    assert np.array_equal(full["T"], again["T"]) and np.array_equal(full["T"], blocked["T"])
    assert full["count"] == again["count"] == blocked["count"] == a["count"] + b["count"]


def test_two_sided_and_identity_gd():
    X, Y = _pair(80, 90, 48, kx=1.5, ky=2.5, seed=14)
    for alt in ["two-sided", "greater"]:
        for gd in ["identity", "banerjee"]:
            r = hbt.perm_test(_dev(X), _dev(Y), 400, seed=3, precision="f32", alternative=alt, gd=gd)
            o = O.perm_test(X, Y, 400, seed=3, alternative=O.ALT_TWO_SIDED if alt != "greater" else 0,
                            gd=O.GD_IDENTITY if gd == "identity" else 0, want_T=True)
            assert r["count"] == o["count"], (alt, gd)


def test_naive_alignment_flag():
    X, Y = _pair(60, 70, 40, seed=15)
    r = hbt.perm_test(_dev(X), _dev(Y), 300, precision="f32", align=False, want_T=True)
    o = O.perm_test(X, Y, 300, align=0, want_T=True)
    assert r["h_identity"] == 1 and r["count"] == o["count"]


def test_no_recheck_flag_counts_raw_precision():
    X, Y = _pair(300, 300, 128, kx=2.0, ky=2.0, seed=16)
    r = hbt.perm_test(_dev(X), _dev(Y), 2000, precision="bf16x2", recheck=False, want_T=True)
    assert r["n_recheck"] == 0
    thr = r["t_obs"] - r["tau"]
    # T_out is rounded to float32, so decisions right at the threshold may differ by a few
    assert abs(r["count"] - int(np.sum(r["T"].astype(np.float64) >= thr))) <= 2


def test_i8x3_equals_exact_sums_of_rounded_rows():
    """The int8 digit planes hold round(z 2^20) exactly and their products with
    the masks are summed in integers, so without the FP64 recheck each T_b is
    the statistic of the rounded rows' sum over the smaller group, and of t
    minus that sum for the larger one, up to FP64 rounding."""
    for n, m, d in [(90, 200, 256), (203, 61, 100)]:
        B = 150
        X, Y = _pair(n, m, d, seed=31 + n)
        r = hbt.perm_test(_dev(X), _dev(Y), B, seed=4, precision="i8x3", recheck=False, want_T="f64")
        a = O.align(X, Y)
        Z = np.vstack([a["Xp"], Y.astype(np.float64)])
        Zq = np.rint(Z * 2.0 ** 20) / 2.0 ** 20
        t = Z.sum(0)
        N = n + m
        T = np.empty(B)
        for b in range(B):
            g1 = O.mask_to_bool(O.split_mask(4, 0, b, N, n), N)
            if n <= m:
                s1 = Zq[g1].sum(0)
                s2 = t - s1
            else:
                s2 = Zq[~g1].sum(0)
                s1 = t - s2
            T[b] = O.log_g(np.linalg.norm(s2) / m, d) - O.log_g(np.linalg.norm(s1) / n, d)
        assert np.abs(r["T"] - T).max() <= 1e-9, (n, m, np.abs(r["T"] - T).max())


def test_i8x3_rejects_point_to_centroid_route():
    X, Y = _pair(20, 30, 16, seed=32)
    with pytest.raises(RuntimeError, match="route 0 only"):
        hbt.perm_test(_dev(X), _dev(Y), 10, precision="i8x3", stat_route=1)


# --------------------------------------------------------------------- point-to-centroid route

@pytest.mark.parametrize("n,m,d,prec", [(37, 150, 100, "f32"), (150, 37, 100, "bf16x2"),
                                        (300, 450, 768, "bf16x2"), (61, 70, 64, "f64"),
                                        (101, 157, 8192, "f32")])
def test_point_to_centroid_route_matches_oracle(n, m, d, prec):
    print(f"route 2 n={n} m={m} d={d} {prec}", flush=True)
    X, Y = _pair(n, m, d, kx=2.0, ky=2.1, seed=n + 3 * m + d)
    B = 700
    r1 = hbt.perm_test(_dev(X), _dev(Y), B, seed=7, precision=prec, want_T="f64")
    r2 = hbt.perm_test(_dev(X), _dev(Y), B, seed=7, precision=prec, stat_route=1, want_T="f64")
    o = O.perm_test(X, Y, B, seed=7, want_T=True)
    at = O.perm_stats_at(X, Y, np.arange(B), seed=7)
    sc = _scale(X, Y, at)
    # route 2 reduces the same norms through FP32 products (FP32 / FP64 first
    # product) or split-BF16 products in three terms: the bar of the precision
    bar = 1e-5 if prec in ("f32", "f64") else TOL[prec]
    assert (np.abs(r2["T"] - o["T"]) / sc).max() <= bar
    assert (np.abs(r2["T"] - r1["T"]) / sc).max() <= 2 * bar
    assert r2["count"] == r1["count"] == o["count"]


@pytest.mark.parametrize("prec", ["f32", "bf16x2", "f64"])
def test_batched_point_to_centroid_route_matches_oracle(prec):
    """The batched call by route 2 (pairs of different sizes and budgets,
    one pair sharing another's splits): counts equal to the oracle's and to
    route 0, moments within the precision's bar."""
    print(f"batched route 2 {prec}", flush=True)
    rng = np.random.default_rng(41)
    pairs = []
    for p in range(9):
        n, m = int(rng.integers(2, 700)), int(rng.integers(2, 700))
        X, Y = _pair(n, m, 200, kx=rng.uniform(1.5, 3), ky=rng.uniform(1.5, 3), seed=300 + p)
        pairs.append(synth.Pair(X, Y, B=int(rng.integers(1, 900)), pair_index=p))
    pairs[5] = synth.Pair(pairs[2].X, pairs[2].Y, B=pairs[2].B, pair_index=2)  # shares pair 2's splits
    bt = synth.pack_batch(pairs, 200)
    args = (_dev(bt.Z), bt.row_offset, bt.n, bt.m, bt.B)
    r2 = hbt.perm_test_batched(*args, seed=9, pair_index=bt.pair_index, precision=prec, stat_route=1)
    r0 = hbt.perm_test_batched(*args, seed=9, pair_index=bt.pair_index, precision=prec)
    for p, pr in enumerate(pairs):
        o = O.perm_test(pr.X, pr.Y, pr.B, seed=9, pair=pr.pair_index, want_T=True)
        assert r2[p]["status"] == 0
        assert abs(r2[p]["count"] - o["count"]) <= _tie_band(o["T"], o["t_obs"]), (prec, p)
        assert r2[p]["count"] == r0[p]["count"] and r2[p]["p"] == r0[p]["p"]
        at = O.perm_stats_at(pr.X, pr.Y, np.arange(pr.B), seed=9, pair=pr.pair_index)
        bar = "f32" if prec in ("f32", "f64") else prec
        _check_extras(r2[p], o, pr.X.shape[0], pr.Y.shape[0], _scale(pr.X, pr.Y, at), bar)
    with pytest.raises(RuntimeError, match="route 0 only"):
        hbt.perm_test_batched(*args, seed=9, precision="i8x3", stat_route=1)


# --------------------------------------------------------------------- batched

def test_batched_matches_oracle_per_pair():
    rng = np.random.default_rng(17)
    pairs = []
    for p in range(7):
        n = int(rng.integers(2, 400))
        m = int(rng.integers(2, 400))
        X, Y = _pair(n, m, 96, kx=rng.uniform(1.5, 3), ky=rng.uniform(1.5, 3), seed=100 + p)
        pairs.append(synth.Pair(X, Y, B=int(rng.integers(1, 700)), pair_index=p))
    pairs[3] = synth.Pair(pairs[3].X, pairs[3].X.copy(), B=300, pair_index=3)  # identical groups
    bt = synth.pack_batch(pairs, 96)
    for prec in ["f32", "bf16x2", "f64", "i8x3", "bf16e4m3", "bf16lazy"]:
        res = hbt.perm_test_batched(_dev(bt.Z), bt.row_offset, bt.n, bt.m, bt.B, seed=9, precision=prec)
        for p, pr in enumerate(pairs):
            o = O.perm_test(pr.X, pr.Y, pr.B, seed=9, pair=p, want_T=True)
            assert res[p]["status"] == 0
            assert abs(res[p]["t_obs"] - o["t_obs"]) <= 1e-12 * max(1, abs(o["t_obs"]))
            assert abs(res[p]["count"] - o["count"]) <= _tie_band(o["T"], o["t_obs"]), (prec, p)
            assert res[p]["B"] == pr.B
            if p != 3:  # identical groups: r at 1 for many splits is fine, moments are not compared
                at = O.perm_stats_at(pr.X, pr.Y, np.arange(pr.B), seed=9, pair=p)
                _check_extras(res[p], o, pr.X.shape[0], pr.Y.shape[0], _scale(pr.X, pr.Y, at), prec)


@pytest.mark.parametrize("prec", ["f64", "bf16x2"])
def test_batched_fp64_rows_match_oracle_per_pair(prec):
    """FP64 input rows in a batch (the recheck gathers them as doubles; the
    FP64 product's band is too narrow to flag any):
    counts, T_obs and moments against the oracle on the same values."""
    rng = np.random.default_rng(18)
    pairs = []
    for p in range(6):
        n = int(rng.integers(2, 700))
        m = int(rng.integers(2, 700))
        X, Y = _pair(n, m, 80, kx=rng.uniform(1.5, 3), ky=rng.uniform(1.5, 3), seed=200 + p)
        pairs.append(synth.Pair(X, Y, B=int(rng.integers(1000, 2500)), pair_index=p))
    bt = synth.pack_batch(pairs, 80)
    print(f"batched FP64 rows {prec}: {len(pairs)} pairs", flush=True)
    res = hbt.perm_test_batched(torch.from_numpy(bt.Z.astype(np.float64)).to(DEV), bt.row_offset, bt.n, bt.m,
                                bt.B, seed=4, precision=prec)
    if prec == "bf16x2":
        assert int(res["n_recheck"].sum()) > 0
    for p, pr in enumerate(pairs):
        o = O.perm_test(pr.X, pr.Y, pr.B, seed=4, pair=p, want_T=True)
        assert res[p]["status"] == 0
        assert abs(res[p]["t_obs"] - o["t_obs"]) <= 1e-12 * max(1, abs(o["t_obs"]))
        assert abs(res[p]["count"] - o["count"]) <= _tie_band(o["T"], o["t_obs"]), (prec, p)
        at = O.perm_stats_at(pr.X, pr.Y, np.arange(pr.B), seed=4, pair=p)
        _check_extras(res[p], o, pr.X.shape[0], pr.Y.shape[0], _scale(pr.X, pr.Y, at), prec)


@pytest.mark.parametrize("d", [64, 200, 1030, 8192])
def test_batched_storage_group_boundaries(d):
    """The Z storage is written in 32-row groups: the column-sum pass stores the
    groups that hold only Y rows or padding, the reflection the groups that hold
    X rows (the one straddling row n included).  Sizes around every boundary
    of that split (n at, just below and above multiples of 32 and 128, m below
    one group, n + m one below / at / above a 128-row padding boundary), d with
    and without zero columns, each pair against the oracle."""
    sizes = [(2, 2), (32, 5), (31, 33), (33, 31), (64, 64), (96, 31), (127, 1 + 1), (128, 2),
             (129, 127), (130, 126), (200, 55), (7, 250), (256, 256), (95, 161)]
    print(f"storage group boundaries d={d}: {len(sizes)} pairs", flush=True)
    pairs = []
    for p, (n, m) in enumerate(sizes):
        X, Y = _pair(n, m, d, kx=2.0, ky=2.6, angle=50.0, seed=300 + p)
        pairs.append(synth.Pair(X, Y, B=257, pair_index=p))
    bt = synth.pack_batch(pairs, d)
    for prec in ["bf16x2", "i8x3", "f32", "bf16e4m3", "bf16lazy"]:
        res = hbt.perm_test_batched(_dev(bt.Z), bt.row_offset, bt.n, bt.m, bt.B, seed=4, precision=prec)
        for p, pr in enumerate(pairs):
            o = O.perm_test(pr.X, pr.Y, pr.B, seed=4, pair=p, want_T=True)
            assert res[p]["status"] == 0, (prec, p)
            assert abs(res[p]["t_obs"] - o["t_obs"]) <= 1e-12 * max(1, abs(o["t_obs"]))
            assert abs(res[p]["count"] - o["count"]) <= _tie_band(o["T"], o["t_obs"]), (prec, p, sizes[p])
            at = O.perm_stats_at(pr.X, pr.Y, np.arange(pr.B), seed=4, pair=p)
            _check_extras(res[p], o, pr.X.shape[0], pr.Y.shape[0], _scale(pr.X, pr.Y, at), prec)


# --------------------------------------------------------------------- full-size configurations

def test_small_pair_f64():
    c = synth.small_pair_f64()
    r = hbt.perm_test(_dev(c.X), _dev(c.Y), c.B, seed=c.seed, precision="f64", want_T=True)
    o = O.perm_test(c.X, c.Y, c.B, seed=c.seed, want_T=True)
    at = O.perm_stats_at(c.X, c.Y, np.arange(c.B))
    err = np.abs(r["T"] - o["T"]) / _scale(c.X, c.Y, at)
    assert err.max() < 1e-7  # T_out is float32
    assert r["count"] == o["count"] and r["p"] == o["p"]
    assert abs(r["t_obs"] - o["t_obs"]) < 1e-12


@pytest.mark.parametrize("prec", ["f32", "bf16x2"])
def test_pair_d768_point_to_centroid_sampled(prec):
    c = synth.pair_d768()
    r = hbt.perm_test(_dev(c.X), _dev(c.Y), 2000, seed=c.seed, precision=prec, stat_route=1, want_T="f64")
    sample = np.arange(0, 2000, 37)
    at = O.perm_stats_at(c.X, c.Y, sample)
    assert (np.abs(r["T"][sample] - at["T"]) / _scale(c.X, c.Y, at)).max() <= (1e-5 if prec == "f32" else 1e-4)


@pytest.mark.parametrize("prec", ["f32", "bf16x2", "i8x3", "bf16e4m3"])
def test_pair_d768_full_size(prec):
    print(f"pair_d768 {prec}", flush=True)
    c = synth.pair_d768()
    Xd, Yd = _dev(c.X), _dev(c.Y)
    r = hbt.perm_test(Xd, Yd, c.B, seed=c.seed, precision=prec, want_T=True)
    sample = np.unique(np.concatenate([np.arange(0, c.B, 97), [c.B - 1]]))
    at = O.perm_stats_at(c.X, c.Y, sample, want_masks=True)
    m = hbt.perm_test(Xd, Yd, 1, seed=c.seed, perm_offset=int(sample[5]), precision=prec, want_masks=True)
    assert np.array_equal(m["masks"][0], at["masks"][5])
    err = np.abs(r["T"][sample] - at["T"]) / _scale(c.X, c.Y, at)
    assert err.max() <= TOL[prec] + 1.2e-7, err.max()
    o = O.perm_test(c.X, c.Y, c.B, seed=c.seed, want_T=True)
    assert abs(r["count"] - o["count"]) <= _tie_band(o["T"], o["t_obs"])
    assert abs(r["t_obs"] - o["t_obs"]) < 1e-12 * abs(o["t_obs"])


_NULL1024 = {}


@pytest.mark.parametrize("prec", ["f32", "bf16x2", "i8x3", "bf16e4m3"])
def test_null_pair_d1024_full_size(prec):
    """The precision-path workload at its stated size (n 3000, m 2000, d 1024,
    B 20,000, equal concentration): counts against the oracle's full run,
    T_b on sampled splits against the oracle's FP64 values, masks bit-exact."""
    print(f"null_pair_d1024 {prec}", flush=True)
    c = synth.null_pair_d1024()
    if not _NULL1024:
        _NULL1024["o"] = O.perm_test(c.X, c.Y, c.B, seed=c.seed, want_T=True)
        sample = np.unique(np.concatenate([np.arange(0, c.B, 101), [c.B - 1]]))
        _NULL1024["sample"] = sample
        _NULL1024["at"] = O.perm_stats_at(c.X, c.Y, sample, seed=c.seed, want_masks=True)
    o, sample, at = _NULL1024["o"], _NULL1024["sample"], _NULL1024["at"]
    Xd, Yd = _dev(c.X), _dev(c.Y)
    r = hbt.perm_test(Xd, Yd, c.B, seed=c.seed, precision=prec, want_T="f64", want_masks=True)
    assert r["status"] == 0
    assert np.array_equal(r["masks"][sample], at["masks"])
    err = np.abs(r["T"][sample] - at["T"]) / _scale(c.X, c.Y, at)
    assert err.max() <= TOL[prec] + 1.2e-7, err.max()
    assert abs(r["count"] - o["count"]) <= _tie_band(o["T"], o["t_obs"]), (r["count"], o["count"])
    assert abs(r["t_obs"] - o["t_obs"]) < 1e-12 * max(1.0, abs(o["t_obs"]))
    assert r["p"] == (1 + r["count"]) / (c.B + 1)
    print(f"  count {r['count']} (oracle {o['count']}), rechecked {r['n_recheck']}, worst T err {err.max():.2e}")


def test_batch_512_d768_full_size_sampled_pairs():
    """The whole 512-pair batch (d = 768, B = 2000 per pair, 1.05M rows) in
    one call per precision, with tile widths tuned on it first, as the
    throughput measurement runs it; 32 pairs at evenly spaced ranks of the
    pooled size, from the smallest to the largest, are checked against the
    oracle (counts, T_obs, p, moments)."""
    print("batch_512_d768 full size", flush=True)
    b = synth.batch_512_d768()
    Z = _dev(b.Z)
    hbt.tune_batched(Z, b.row_offset, b.n, b.m, b.B, seed=b.seed)
    res = {prec: hbt.perm_test_batched(Z, b.row_offset, b.n, b.m, b.B, seed=b.seed, precision=prec)
           for prec in ["bf16x2", "i8x3", "bf16e4m3", "bf16lazy"]}
    del Z
    order = np.argsort(b.n + b.m, kind="stable")
    P = b.npairs
    # 32 pairs at evenly spaced ranks of the pooled size, smallest and largest included
    picks = sorted(set(np.linspace(0, P - 1, 32).round().astype(int).tolist()))
    assert len(picks) == 32
    for p in (int(order[k]) for k in picks):
        pr = b.pair(p)
        print(f"pair {p}: n={pr.X.shape[0]} m={pr.Y.shape[0]}", flush=True)
        o = O.perm_test(pr.X, pr.Y, pr.B, seed=b.seed, pair=p, want_T=True)
        at = O.perm_stats_at(pr.X, pr.Y, np.arange(0, pr.B, 10), seed=b.seed, pair=p)
        for prec, r in res.items():
            assert np.all(r["status"] == 0), prec
            assert abs(r[p]["t_obs"] - o["t_obs"]) <= 1e-12 * max(1.0, abs(o["t_obs"])), (prec, p)
            assert abs(r[p]["count"] - o["count"]) <= _tie_band(o["T"], o["t_obs"]), (prec, p)
            assert r[p]["B"] == pr.B and r[p]["p"] == (1 + r[p]["count"]) / (pr.B + 1)
            _check_extras(r[p], o, pr.X.shape[0], pr.Y.shape[0], _scale(pr.X, pr.Y, at), prec)


# --------------------------------------------------------------------- graph capture

@pytest.mark.parametrize("prec", ["bf16x2", "bf16lazy"])
def test_batched_call_replays_from_a_hip_graph(prec):
    """The batched call enqueues only kernels on the caller's stream (tables go
    in as kernel arguments, no memset, no allocation, no synchronisation), so
    it can be captured once and replayed.  Every replay, with eager calls that
    reuse the same workspace in between, must reproduce the eager results.
    (The lazy precision's refinement lists and tile table are built on the
    device each call, its counters cleared by a fill kernel.)"""
    print(f"graph capture {prec}: 12 pairs of the 512-pair workload", flush=True)
    b = synth.batch_512_d768(limit=range(12))
    Z = _dev(b.Z)
    args = (Z, b.row_offset, b.n, b.m, b.B)
    ref = hbt.perm_test_batched(*args, seed=b.seed, precision=prec)
    need = hbt.batched_workspace_size(b.row_offset, b.n, b.m, b.B, b.d, precision=prec)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    res = torch.zeros(hbt.RESULT_BYTES * b.npairs, dtype=torch.uint8, device=DEV)
    hbt.perm_test_batched(*args, seed=b.seed, precision=prec, sync=False, results=res, workspace=ws)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hbt.perm_test_batched(*args, seed=b.seed, precision=prec, sync=False, results=res, workspace=ws)
    fields = ["t_obs", "r_x", "r_y", "p", "t_mean", "t_sd", "count", "B", "n_recheck", "status"]
    for rep in range(3):
        res.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = hbt.results_to_numpy(res)
        for f in fields:
            assert np.array_equal(got[f], ref[f]), (rep, f)
        # eager work on the same workspace between replays (another seed)
        other = hbt.perm_test_batched(*args, seed=b.seed + 1, precision=prec, workspace=ws)
        assert np.all(other["status"] == 0)


@pytest.mark.parametrize("prec", ["bf16x2", "i8x3"])
def test_pipeline_chunks_do_not_change_results(prec):
    """The batched call pipelines chunks of pairs over three streams; every
    chunking gives the same results, bit for bit, as one chunk."""
    print(f"pipeline chunks {prec}: 60 pairs of the 512-pair workload", flush=True)
    b = synth.batch_512_d768(limit=range(60))
    Z = _dev(b.Z)
    prev = hbt.pipeline_chunks(1)
    try:
        ref = hbt.perm_test_batched(Z, b.row_offset, b.n, b.m, b.B, seed=b.seed, precision=prec)
        for c in (2, 3, 4, 7, 60):
            hbt.pipeline_chunks(c)
            got = hbt.perm_test_batched(Z, b.row_offset, b.n, b.m, b.B, seed=b.seed, precision=prec)
            _results_equal(got, ref)
    finally:
        hbt.pipeline_chunks(prev)
    assert np.all(ref["status"] == 0)


# --------------------------------------------------------------------- tile widths

def _results_equal(a, b):
    for f in ["t_obs", "r_x", "r_y", "p", "t_mean", "t_sd", "count", "B", "n_recheck", "status"]:
        assert np.array_equal(a[f], b[f]), f


def test_pairs_with_equal_sizes_and_index_share_their_splits():
    """Pairs with equal n, m, B and pair index have the same splits by
    definition (same counters, same key): the batched call draws them once and
    the other pairs read the first one's masks.  Pairs 0, 2, 4 share them
    (different data), pair 5 has the same index but swapped sizes and draws its
    own; every pair must match the oracle run with its pair index."""
    d = 96
    sizes = [(120, 90), (120, 90), (120, 90), (60, 200), (120, 90), (90, 120)]
    index = [7, 1, 7, 3, 7, 7]
    pairs = []
    for p, ((n, m), k) in enumerate(zip(sizes, index)):
        X, Y = _pair(n, m, d, kx=2.0, ky=2.3, angle=30.0, seed=500 + p)
        pairs.append(synth.Pair(X, Y, B=400, pair_index=k))
    bt = synth.pack_batch(pairs, d)
    for prec in ["bf16x2", "f32", "i8x3", "bf16lazy"]:
        res = hbt.perm_test_batched(_dev(bt.Z), bt.row_offset, bt.n, bt.m, bt.B, seed=11,
                                    pair_index=bt.pair_index, precision=prec)
        for p, pr in enumerate(pairs):
            o = O.perm_test(pr.X, pr.Y, pr.B, seed=11, pair=pr.pair_index, want_T=True)
            assert res[p]["status"] == 0, (prec, p)
            assert abs(res[p]["t_obs"] - o["t_obs"]) <= 1e-12 * max(1, abs(o["t_obs"]))
            assert abs(res[p]["count"] - o["count"]) <= _tie_band(o["T"], o["t_obs"]), (prec, p)
            at = O.perm_stats_at(pr.X, pr.Y, np.arange(pr.B), seed=11, pair=pr.pair_index)
            _check_extras(res[p], o, pr.X.shape[0], pr.Y.shape[0], _scale(pr.X, pr.Y, at), prec)


def test_recheck_value_does_not_depend_on_how_it_is_spread(monkeypatch):
    """A flagged split's FP64 group sum is formed in one order: per wave its
    rows of a 512-row segment in ascending order, the segment's wave sums in
    wave order, the segments in order.  The benchmark batch takes its flags
    segment by segment (one work item per flag and segment, the segment sums
    added by a second kernel); with HBT_RECHECK_SLOTS=0 every flag is one
    work item over all its segments, and with 2000 slots the first pairs are
    done one way and the rest the other; a single-pair call takes its few
    flags segment by segment.  Counts, n_recheck and the null moments (which
    hold the rechecked T_b) must agree bit for bit."""
    b = synth.batch_512_d768()
    print(f"recheck spread: {b.npairs} pairs of the 512-pair workload", flush=True)
    Z = _dev(b.Z)
    res = hbt.perm_test_batched(Z, b.row_offset, b.n, b.m, b.B, seed=b.seed, precision="bf16x2")
    assert int(res["n_recheck"].sum()) >= 1000  # more flag segments than 2000 slots
    # 0 slots: every flag whole; 2000 slots: the first pairs' flags by
    # segment, the others whole, in the same call
    for slots in ["0", "2000"]:
        monkeypatch.setenv("HBT_RECHECK_SLOTS", slots)
        other = hbt.perm_test_batched(Z, b.row_offset, b.n, b.m, b.B, seed=b.seed, precision="bf16x2")
        for f in ["count", "n_recheck", "t_mean", "t_sd", "status"]:
            assert np.array_equal(other[f], res[f]), (slots, f)
    monkeypatch.delenv("HBT_RECHECK_SLOTS")
    del Z
    checked = 0
    for p in np.nonzero(res["n_recheck"] > 1)[0][:8]:
        pr = b.pair(int(p))
        one = hbt.perm_test(_dev(pr.X), _dev(pr.Y), pr.B, seed=b.seed, pair_index=pr.pair_index,
                            precision="bf16x2")
        for f in ["t_obs", "count", "p", "n_recheck", "t_mean", "t_sd"]:
            assert one[f] == res[p][f], (int(p), f, one[f], res[p][f])
        checked += 1
    assert checked > 0
    # a single pair of ten segments: its flags by segment, or each whole
    pr = synth.null_pair_d1024()
    X, Y = _dev(pr.X), _dev(pr.Y)
    seg = hbt.perm_test(X, Y, pr.B, seed=pr.seed, precision="bf16x2", want_T="f64")
    monkeypatch.setenv("HBT_RECHECK_SLOTS", "0")
    whole = hbt.perm_test(X, Y, pr.B, seed=pr.seed, precision="bf16x2", want_T="f64")
    monkeypatch.delenv("HBT_RECHECK_SLOTS")
    assert seg["n_recheck"] > 0
    for f in ["count", "n_recheck", "t_mean", "t_sd", "status"]:
        assert whole[f] == seg[f], f


def test_single_pair_wide_and_narrow_tiles_agree():
    """A single-pair call takes the wide tile only when it gives at least two
    tiles per CU; this pair (d = 1024, 32768 splits: 32 x 16 wide tiles) does,
    so the call runs the eight-wave kernel with wide costs and the narrow one
    with narrow costs, and the results must agree bit for bit."""
    d, B = 1024, 32768
    X, Y = _pair(300, 420, d, kx=2.0, ky=2.1, seed=71)
    Xd, Yd = _dev(X), _dev(Y)
    saved, _ = hbt.tune_get(d)
    try:
        runs = []
        for costs in [(1.0, 1e9), (1e9, 1.0)]:
            hbt.tune_set(d, costs)
            runs.append(hbt.perm_test(Xd, Yd, B, seed=3, precision="bf16x2", want_T="f64"))
    finally:
        hbt.tune_set(d, saved)
    assert runs[0]["status"] == 0 and runs[1]["status"] == 0
    assert np.array_equal(runs[0]["T"], runs[1]["T"])
    for k in ["t_obs", "count", "p", "n_recheck", "t_mean", "t_sd"]:
        assert runs[0][k] == runs[1][k], k
    o = O.perm_test(X, Y, 200, seed=3, want_T=True)  # the first 200 splits against the oracle
    err = np.abs(runs[0]["T"][:200] - o["T"]) / _scale(X, Y, O.perm_stats_at(X, Y, np.arange(200), seed=3))
    assert err.max() <= TOL["bf16x2"], err.max()


def test_tile_widths_do_not_change_results():
    """The product runs per pair with 1024- or 256-split tiles; each split's
    sums come from the same instructions in the same order, so results are
    bit-identical whichever width the table picks."""
    rng = np.random.default_rng(23)
    pairs = []
    for p in range(6):
        n, m = int(rng.integers(2, 500)), int(rng.integers(2, 500))
        X, Y = _pair(n, m, 160, kx=rng.uniform(1.5, 3), ky=rng.uniform(1.5, 3), seed=300 + p)
        pairs.append(synth.Pair(X, Y, B=int(rng.integers(1, 1300)), pair_index=p))
    bt = synth.pack_batch(pairs, 160)
    runs = []
    for costs in [(1.0, 1e9), (1e9, 1.0)]:
        hbt.tune_set(160, costs)
        assert set(hbt.tile_widths(bt.B, 160)) == ({1024} if costs[0] < costs[1] else {256})
        runs.append(hbt.perm_test_batched(_dev(bt.Z), bt.row_offset, bt.n, bt.m, bt.B, seed=4,
                                          precision="bf16x2"))
        X, Y = pairs[0].X, pairs[0].Y
        runs.append(hbt.perm_test(_dev(X), _dev(Y), 1100, seed=4, precision="bf16x2", want_T="f64"))
    hbt.tune_set(160, (1.0, 1.15))
    _results_equal(runs[0], runs[2])
    assert np.array_equal(runs[1]["T"], runs[3]["T"])
    for k in ["t_obs", "count", "p", "t_mean", "t_sd"]:
        assert runs[1][k] == runs[3][k]


def test_tuning_measures_both_widths():
    b = synth.batch_512_d768(limit=range(24))
    costs = hbt.tune_batched(_dev(b.Z), b.row_offset, b.n, b.m, np.full(24, 300))
    (c1024, c256), tuned = hbt.tune_get(768)
    assert tuned and c1024 > 0 and c256 > 0 and (c1024, c256) == costs
    print(f"tuned per-split costs at d=768: 1024-wide {c1024:.3e}, 256-wide {c256:.3e} ms", flush=True)
    Bs = [1, 256, 300, 1024, 2000, 5000]
    up = lambda B, w: -(-B // w) * w
    want = [256 if c256 * up(B, 256) < c1024 * up(B, 1024) else 1024 for B in Bs]
    assert list(hbt.tile_widths(Bs, 768)) == want


@pytest.mark.parametrize("prec", ["bf16x2", "i8x3"])
def test_tuner_picks_launch_parameters_from_its_candidates(prec, tmp_path):
    """The tuner measures grids, split work-groups per CU and pipeline chunks
    and installs them; the tuned calls give the untuned results; the entry
    round-trips through the JSON cache."""
    print(f"tuner {prec}", flush=True)
    b = synth.batch_512_d768(limit=range(40))
    Z = _dev(b.Z)
    d = 768
    before = hbt.tune_entry_get(prec, d)
    ref = hbt.perm_test_batched(Z, b.row_offset, b.n, b.m, b.B, seed=b.seed, precision=prec)
    try:
        hbt.tune_batched(Z, b.row_offset, b.n, b.m, b.B, seed=b.seed, precision=prec)
        e = hbt.tune_entry_get(prec, d)
        print(f"  tuned: {e}", flush=True)
        assert e["tuned"] and e["grid_wide"] in (4, 8, 16, 32) and e["grid_narrow"] in (8, 16, 32, 64)
        assert e["split_cap"] in (4, 5, 6, 8) and e["chunks"] in (1, 2, 4)
        _results_equal(hbt.perm_test_batched(Z, b.row_offset, b.n, b.m, b.B, seed=b.seed, precision=prec), ref)
        f = tmp_path / "tune.json"
        hbt.save_tuning(f)
        hbt.tune_entry_set(prec, d, dict(before, cost=(1.0, 1.15)))
        hbt.load_tuning(f)
        assert hbt.tune_entry_get(prec, d) == e
    finally:
        hbt.tune_entry_set(prec, d, before)

