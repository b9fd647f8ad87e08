"""The FP64 recheck band against an exact emulation of the stored rows (CPU).

A split is re-evaluated in FP64 when its reduced-precision T_b lies within the
library's band (hbt_recheck_band) of the threshold, so the band must cover
|T_b - T_b(FP64)| for every split, or a split could be decided on the wrong
side without a recheck.  Here the rows are stored as the kernels store them
(FP32; split BF16 hi = bf16(z), lo = bf16(z - hi), both round-to-nearest-even
from the FP32 row; BF16 + e4m3 the same hi and lo = e4m3(2^17 (z - hi)) 2^-17,
nearest-even; int8 digits of round(z 2^20) from the FP64 row; the lazy
precision's first pass the hi plane alone) and the
group sums are formed exactly in FP64, which isolates the storage error
(the accumulation error is the band's e_acc, checked on the GPU).

The hard cases are clouds whose rows repeat (the same sentence many times
gives identical vectors, so the rounding errors of a group sum add up
coherently instead of averaging out) and diffuse clouds (r ~ 0.02-0.05, where
a fixed error of the sum is large relative to its norm).  The bar is half the
band; the emulated worst case with the shipped constants is about a quarter.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_08048_amd import hbt, synth


def _bf16(a):
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _e4m3(x):
    """Nearest e4m3 value (OCP E4M3FN: 4 significant bits, smallest normal
    2^-6, subnormal spacing 2^-9), ties to even; |x| <= 448 here."""
    x = np.asarray(x, np.float64)
    a = np.abs(x)
    _, E = np.frexp(np.where(a > 0, a, 1.0))        # a = f 2^E, f in [0.5, 1)
    q = np.where(a < 2.0 ** -6, 2.0 ** -9, np.ldexp(1.0, E - 4))  # spacing of a's binade
    return np.sign(x) * np.rint(a / q) * q


def _stored(Z, prec):
    if prec == "i8x3":
        return np.rint(Z * 2.0 ** 20) / 2.0 ** 20
    zf = Z.astype(np.float32)
    if prec == "f32":
        return zf.astype(np.float64)
    hi = _bf16(zf)
    if prec == "bf16lazy":  # the lazy precision's first pass: the hi plane alone
        return hi.astype(np.float64)
    if prec == "bf16e4m3":
        lo = (zf - hi).astype(np.float64)            # exact in FP32
        return hi.astype(np.float64) + _e4m3(lo * 2.0 ** 17) / 2.0 ** 17
    lo = _bf16(zf - hi)
    return hi.astype(np.float64) + lo.astype(np.float64)


def test_e4m3_rounding_definition():
    """The emulation's e4m3 grid: exact values stay, ties go to the even
    significand, subnormals step by 2^-9."""
    v = np.array([1.0, 1.125, 1.0625, 1.1875, 448.0, 2.0 ** -6, 2.0 ** -9, 3 * 2.0 ** -10, 2.0 ** -10, 0.0, -1.0625])
    want = np.array([1.0, 1.125, 1.0, 1.25, 448.0, 2.0 ** -6, 2.0 ** -9, 2 * 2.0 ** -9, 0.0, 0.0, -1.0])
    assert np.array_equal(_e4m3(v), want)


def _cloud(g, n, d, kappa, mu, rep):
    """n unit rows around mu, made of n // rep distinct rows repeated rep times
    in random order."""
    k = max(1, n // rep)
    base = synth.unit_rows(kappa * mu + g.standard_normal((k, d)) / math.sqrt(d))
    idx = np.concatenate([np.arange(k)] * (n // k + 1))[:n]
    g.shuffle(idx)
    return base[idx].astype(np.float32)


def _worst_ratio(n, m, d, kx, ky, rep, B, seed=0):
    g = np.random.default_rng([9, seed, n, m, d, rep])
    mu = synth.random_unit(g, d)
    mv = synth.direction_at_angle(g, mu, 40.0)
    X = _cloud(g, n, d, kx, mu, rep)
    Y = _cloud(g, m, d, ky, mv, rep)
    a = O.align(X, Y)
    Z = np.vstack([a["Xp"], Y.astype(np.float64)])
    N = n + m
    t = Z.sum(0)
    M = np.zeros((B, N))
    for b in range(B):
        M[b, g.permutation(N)[:n]] = 1.0
    small1 = n <= m
    Ms = M if small1 else 1.0 - M

    def stat(Zs):
        s_small = Ms @ Zs
        s_large = t - s_small
        s1, s2 = (s_small, s_large) if small1 else (s_large, s_small)
        r1 = np.linalg.norm(s1, axis=1) / n
        r2 = np.linalg.norm(s2, axis=1) / m
        f = np.vectorize(lambda r: O.log_g(r, d))
        return r1, r2, f(r2) - f(r1)

    r1, r2, T64 = stat(Z)
    out = {}
    # the lazy precision's first pass decides nothing for pairs with a group
    # under 16 items (every split goes to the split-BF16 product)
    lazy = ("bf16lazy",) if min(n, m) >= 16 else ()
    for prec in ("f32", "bf16x2", "i8x3", "bf16e4m3") + lazy:
        T = stat(_stored(Z, prec))[2]
        eps = hbt.recheck_band(prec, n, m, d, r1, r2)
        out[prec] = float((np.abs(T - T64) / eps).max())
    return float(np.median(r1)), out


CASES = [
    # n, m, d, kappa_x, kappa_y, repeats, splits
    (1000, 1000, 768, 2.0, 2.4, 1, 200),
    (1000, 1000, 768, 2.0, 2.4, 10, 200),
    (1000, 1000, 768, 2.0, 2.4, 100, 200),
    (1000, 1000, 768, 2.0, 2.4, 500, 200),
    (4000, 4000, 1024, 2.0, 2.4, 1000, 100),
    (1000, 1000, 768, 0.03, 0.03, 1, 200),     # diffuse, r ~ 0.05
    (3000, 2000, 1024, 0.02, 0.02, 1, 100),    # diffuse, r ~ 0.03
    (3000, 2000, 1024, 0.02, 0.02, 100, 100),
    (1000, 1000, 768, 0.03, 0.03, 500, 200),
    (2, 300, 64, 8.0, 8.0, 1, 300),            # a group of 2, r near 1
    (300, 2, 64, 0.05, 0.05, 1, 300),
    (20, 5000, 768, 0.05, 0.05, 10, 200),
    (5000, 20, 768, 2.0, 2.0, 10, 200),
    (900, 1100, 768, 30.0, 30.0, 300, 200),    # r ~ 0.9995, repeated rows
    (2, 2000, 768, 0.05, 0.05, 1, 300),        # a group of 2 in a diffuse cloud
    (100, 100, 64, 8.0, 8.0, 50, 100),
    (16, 300, 64, 8.0, 8.0, 1, 300),           # the smallest groups the lazy first pass decides
    (300, 16, 64, 0.05, 0.05, 1, 300),
    (16, 16, 64, 8.0, 8.0, 1, 300),
]
SEEDS = {1: [0], 10: [0]}  # repeated rows: the worst case depends on which rows repeat


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n{}_m{}_d{}_k{}_rep{}".format(*c[:4], c[5]))
def test_stored_rows_stay_inside_the_recheck_band(case):
    n, m, d, kx, ky, rep, B = case
    for seed in SEEDS.get(rep, range(4)):
        r, worst = _worst_ratio(n, m, d, kx, ky, rep, B, seed=seed)
        print(f"n={n} m={m} d={d} rep={rep} seed={seed} r1~{r:.3f} worst |T - T64| / band: "
              + ", ".join(f"{k} {v:.3f}" for k, v in worst.items()))
        for prec, ratio in worst.items():
            assert ratio <= 0.5, (prec, case, seed, ratio)


def test_band_grows_for_diffuse_groups_and_repeats_nothing_over_k():
    """The storage term does not shrink with the group size (rows may repeat)
    and grows as 1/r; the route-2 band is at least the FP32 one."""
    b = lambda prec, n, r, route=0: hbt.recheck_band(prec, n, n, 768, r, r, stat_route=route)
    assert b("i8x3", 4000, 0.9) >= 0.99 * b("i8x3", 100, 0.9)
    assert b("i8x3", 1000, 0.02) > 10 * b("i8x3", 1000, 0.5) * 0.5 / 0.02 * 0.02 / 0.5
    assert b("f64", 1000, 0.5, 1) >= b("f32", 1000, 0.5, 0)
    assert b("bf16x2", 1000, 0.5, 1) > b("bf16x2", 1000, 0.5, 0)
    assert hbt.recheck_band("f32", 50, 60, 8192, 0.3, 0.3, stat_route=1) > \
        hbt.recheck_band("f32", 50, 60, 64, 0.3, 0.3, stat_route=1)
    with pytest.raises(hbt.HbtError):
        hbt.recheck_band("f32", 0, 60, 64, 0.3, 0.3)
