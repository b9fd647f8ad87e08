"""Seeded synthetic inputs: clouds of unit vectors on the sphere S^{d-1}.

This module is shared by the tests, the benchmark and the smoke check.  It
holds no arithmetic of the test itself (no means, no reflection, no
statistic): it only draws anisotropic Gaussian noise around a mean direction
and projects each row onto the unit sphere, the normalisation the paper
applies to every token embedding before testing (Sec. 3.1, Eq. 2).

Every array is reproducible from integers alone:
``numpy.random.default_rng(SeedSequence([stream, pair, side]))``, with one
stream number per workload.

Workloads (stand-ins for BERT-family token embeddings of corpus words, which
are not available here; shapes follow the paper's d = 768 / 1024 encoders and
its B = 5,000 ... 20,000 permutation budgets):

* small_pair_f64 (stream 1) - one pair, d=64, n=50, m=60, diagonal noise lambda_i ~ 1/i
  (trace 1), kappa = 3, independent mean directions, FP64.
* pair_d768 (stream 2) - one pair, d=768, n=2000, m=1500, low-rank noise, kappa 2.0/2.4,
  means 40 degrees apart, FP32.
* null_pair_d1024 (stream 3) - one pair, d=1024, n=3000, m=2000, low-rank noise, equal
  kappa = 2.2 (null), FP32 input for the split-BF16 path.
* batch_512_d768 (stream 4) - 512 pairs, d=768, n_p and m_p log-uniform on [20, 5000],
  kappa ~ U[1.5, 3.0], half the pairs null, random mean directions.
* budget_batch_4096 (stream 5) - 4096 pairs, d=768, n and m log-uniform on [20, 2000].
* rejection_batch (stream 6) - the shape of the paper's rejection-rate experiment:
  500 pairs, d=768, B=5000; n log-uniform on [100, 1000] and m within 10% of n,
  kappa_X ~ U[2, 4], mean directions U[20, 70] degrees apart; "null" keeps
  kappa_Y = kappa_X, "alt" makes Y 2% more concentrated (X broader).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng_for", "unit_rows", "random_unit", "direction_at_angle", "lowrank_factor",
    "cloud_diag", "cloud_lowrank", "Pair", "Batch", "small_pair_f64", "pair_d768", "null_pair_d1024",
    "batch_512_d768", "budget_batch_4096", "rejection_batch", "pack_batch", "log_uniform_int",
]


def rng_for(stream: int, pair: int = 0, side: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(stream), int(pair), int(side)]))


def unit_rows(a: np.ndarray) -> np.ndarray:
    """Project each row onto the unit sphere (computed in float64)."""
    a = np.asarray(a, dtype=np.float64)
    return a / np.linalg.norm(a, axis=-1, keepdims=True)


def random_unit(rng: np.random.Generator, d: int) -> np.ndarray:
    return unit_rows(rng.standard_normal(d))


def direction_at_angle(rng: np.random.Generator, mu: np.ndarray, degrees: float) -> np.ndarray:
    """A unit vector at the given angle from the unit vector ``mu``."""
    w = rng.standard_normal(mu.shape[0])
    w -= (w @ mu) * mu
    w /= np.linalg.norm(w)
    a = math.radians(degrees)
    return math.cos(a) * mu + math.sin(a) * w


def lowrank_factor(d: int, rank: int = 32, seed: int = 1, noise: float = 0.1):
    """Fixed noise model Sigma = s^2 (L L^T + noise^2 I), scaled to unit trace.

    Returns (L, noise, s).  A draw is w = s * (L z1 + noise * z2).
    """
    g = np.random.default_rng(np.random.SeedSequence([1000, int(d), int(rank), int(seed)]))
    L = g.standard_normal((d, rank)) / math.sqrt(rank)
    trace = float(np.sum(L * L)) + noise * noise * d
    return L, noise, 1.0 / math.sqrt(trace)


def cloud_diag(rng, n, d, kappa, mu, lam):
    """x = normalize(kappa * mu + z), z ~ N(0, diag(lam))."""
    z = rng.standard_normal((n, d)) * np.sqrt(lam)[None, :]
    return unit_rows(kappa * mu[None, :] + z)


def cloud_lowrank(rng, n, d, kappa, mu, factor):
    """x = normalize(kappa * mu + s (L z1 + noise z2)); z1, z2 drawn in float32."""
    L, noise, s = factor
    z1 = rng.standard_normal((n, L.shape[1]), dtype=np.float32)
    z2 = rng.standard_normal((n, d), dtype=np.float32)
    w = (z1 @ L.T.astype(np.float32) + np.float32(noise) * z2).astype(np.float64) * s
    return unit_rows(kappa * mu[None, :] + w)


@dataclass
class Pair:
    X: np.ndarray            # (n, d) unit rows
    Y: np.ndarray            # (m, d) unit rows
    B: int                   # permutations
    seed: int = 0            # permutation seed
    pair_index: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def m(self):
        return self.Y.shape[0]

    @property
    def d(self):
        return self.X.shape[1]


def small_pair_f64() -> Pair:
    d, n, m = 64, 50, 60
    lam = 1.0 / np.arange(1, d + 1)
    lam /= lam.sum()
    mu_a = random_unit(rng_for(1, 0, 10), d)
    mu_b = random_unit(rng_for(1, 0, 11), d)
    X = cloud_diag(rng_for(1, 0, 0), n, d, 3.0, mu_a, lam)
    Y = cloud_diag(rng_for(1, 0, 1), m, d, 3.0, mu_b, lam)
    return Pair(X, Y, B=999, seed=0, meta=dict(workload="small_pair_f64", dtype="f64"))


def _lowrank_pair(stream, pair, n, m, d, kappa_a, kappa_b, angle=None, factor=None):
    factor = factor if factor is not None else lowrank_factor(d)
    mu_a = random_unit(rng_for(stream, pair, 10), d)
    if angle is None:
        mu_b = random_unit(rng_for(stream, pair, 11), d)
    else:
        mu_b = direction_at_angle(rng_for(stream, pair, 11), mu_a, angle)
    X = cloud_lowrank(rng_for(stream, pair, 0), n, d, kappa_a, mu_a, factor)
    Y = cloud_lowrank(rng_for(stream, pair, 1), m, d, kappa_b, mu_b, factor)
    return X.astype(np.float32), Y.astype(np.float32)


def pair_d768(n=2000, m=1500, d=768, B=10000) -> Pair:
    X, Y = _lowrank_pair(2, 0, n, m, d, 2.0, 2.4, angle=40.0)
    return Pair(X, Y, B=B, seed=0, meta=dict(workload="pair_d768", dtype="f32"))


def null_pair_d1024(n=3000, m=2000, d=1024, B=20000) -> Pair:
    X, Y = _lowrank_pair(3, 0, n, m, d, 2.2, 2.2, angle=40.0)
    return Pair(X, Y, B=B, seed=0, meta=dict(workload="null_pair_d1024", dtype="f32"))


def log_uniform_int(rng, lo, hi, size=None):
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi + 1), size=size))).astype(np.int64).clip(lo, hi)


@dataclass
class Batch:
    Z: np.ndarray            # (sum_p n_p + m_p, d) float32: X_0, Y_0, X_1, Y_1, ...
    row_offset: np.ndarray   # (P+1,) int64, row of X_p
    n: np.ndarray            # (P,) int64
    m: np.ndarray            # (P,) int64
    B: np.ndarray            # (P,) int64
    pair_index: np.ndarray = None  # (P,) uint32 Philox counter word per pair
    seed: int = 0
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.pair_index is None:
            self.pair_index = np.arange(self.n.shape[0], dtype=np.uint32)

    @property
    def npairs(self):
        return int(self.n.shape[0])

    @property
    def d(self):
        return int(self.Z.shape[1])

    def pair(self, p) -> Pair:
        o = int(self.row_offset[p])
        n, m = int(self.n[p]), int(self.m[p])
        return Pair(self.Z[o:o + n], self.Z[o + n:o + n + m], B=int(self.B[p]), seed=self.seed,
                    pair_index=int(self.pair_index[p]))


def pack_batch(pairs, d, seed=0, meta=None) -> Batch:
    n = np.array([p.X.shape[0] for p in pairs], dtype=np.int64)
    m = np.array([p.Y.shape[0] for p in pairs], dtype=np.int64)
    B = np.array([p.B for p in pairs], dtype=np.int64)
    off = np.zeros(len(pairs) + 1, dtype=np.int64)
    off[1:] = np.cumsum(n + m)
    Z = np.empty((int(off[-1]), d), dtype=np.float32)
    for i, p in enumerate(pairs):
        Z[off[i]:off[i] + n[i]] = p.X
        Z[off[i] + n[i]:off[i + 1]] = p.Y
    ids = np.array([p.pair_index for p in pairs], dtype=np.uint32)
    return Batch(Z, off, n, m, B, pair_index=ids, seed=seed, meta=meta or {})


def _batch_workload(stream, npairs, d, lo, hi, B, limit=None):
    g = rng_for(stream, 0, 99)
    ns = log_uniform_int(g, lo, hi, npairs)
    ms = log_uniform_int(g, lo, hi, npairs)
    ka = g.uniform(1.5, 3.0, npairs)
    kb = g.uniform(1.5, 3.0, npairs)
    null = np.arange(npairs) % 2 == 0
    kb = np.where(null, ka, kb)
    factor = lowrank_factor(d)
    idx = list(range(npairs) if limit is None else limit)

    def one(p):
        X, Y = _lowrank_pair(stream, p, int(ns[p]), int(ms[p]), d, float(ka[p]), float(kb[p]),
                             angle=None, factor=factor)
        return Pair(X, Y, B=B, seed=0, pair_index=p, meta=dict(null=bool(null[p])))

    # every pair has its own seeded generator, so the thread pool changes nothing
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        pairs = list(ex.map(one, idx))
    return pairs, dict(kappa_a=ka, kappa_b=kb, null=null, n=ns, m=ms)


def batch_512_d768(npairs=512, d=768, B=2000, limit=None) -> Batch:
    pairs, info = _batch_workload(4, npairs, d, 20, 5000, B, limit)
    return pack_batch(pairs, d, meta=dict(workload="batch_512_d768", **info))


def budget_batch_4096(npairs=4096, d=768, B=20000, limit=None) -> Batch:
    pairs, info = _batch_workload(5, npairs, d, 20, 2000, B, limit)
    return pack_batch(pairs, d, meta=dict(workload="budget_batch_4096", **info))


REJECTION_EFFECT = 0.02


def rejection_batch(population="null", npairs=500, d=768, B=5000, limit=None) -> Batch:
    """Pairs shaped like the paper's rejection-rate experiment (Sec. 5 of the
    appendix experiments: 500 word pairs, B = 5,000, alpha = 0.05, a null and an
    alternative condition).

    Words a few frequency ranks apart have similar token counts, so m is drawn
    within 10% of n.  Both conditions give the two clouds different mean
    directions (the confounder the alignment removes); "null" keeps the same
    breadth, "alt" makes Y's cloud more concentrated by REJECTION_EFFECT in
    kappa, so X is the broader one and the "greater" alternative holds.  The two
    conditions share every draw except kappa_Y (common random numbers), so their
    rates are compared on the same clouds and directions.
    """
    if population not in ("null", "alt"):
        raise ValueError("population must be 'null' or 'alt'")
    g = rng_for(6, 0, 99)
    ns = log_uniform_int(g, 100, 1000, npairs)
    ms = np.rint(ns * g.uniform(0.9, 1.1, npairs)).astype(np.int64)
    ka = g.uniform(2.0, 4.0, npairs)
    angle = g.uniform(20.0, 70.0, npairs)
    kb = ka * (1.0 + (REJECTION_EFFECT if population == "alt" else 0.0))
    factor = lowrank_factor(d)
    idx = list(range(npairs) if limit is None else limit)

    def one(p):
        X, Y = _lowrank_pair(6, p, int(ns[p]), int(ms[p]), d, float(ka[p]), float(kb[p]),
                             angle=float(angle[p]), factor=factor)
        return Pair(X, Y, B=B, seed=0, pair_index=p)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        pairs = list(ex.map(one, idx))
    return pack_batch(pairs, d, meta=dict(workload="rejection_batch", population=population,
                                          kappa_a=ka, kappa_b=kb, angle=angle, n=ns, m=ms))


@dataclass
class Clouds:
    Z: np.ndarray            # (sum of cloud rows, d) float32
    offset: np.ndarray       # (C,) int64 first row of each cloud
    rows: np.ndarray         # (C,) int64
    pair_x: np.ndarray       # (P,) int64 cloud of X
    pair_y: np.ndarray       # (P,) int64 cloud of Y
    B: np.ndarray            # (P,) int64
    seed: int = 0
    meta: dict = field(default_factory=dict)

    def pairs_batch(self) -> Batch:
        """The same pairs packed one by one (rows X_0, Y_0, X_1, ...)."""
        o, r = self.offset, self.rows
        pairs = [Pair(self.Z[o[x]:o[x] + r[x]], self.Z[o[y]:o[y] + r[y]], B=int(b), pair_index=p)
                 for p, (x, y, b) in enumerate(zip(self.pair_x, self.pair_y, self.B))]
        return pack_batch(pairs, self.Z.shape[1], seed=self.seed)


def word_clouds(nwords=64, npairs=512, d=768, lo=20, hi=5000, B=2000) -> Clouds:
    """Words whose clouds take part in many pairs (each word in about
    2 npairs / nwords of them): a cloud per word, n log-uniform on [lo, hi],
    kappa ~ U[1.5, 3], a random mean direction; pairs of distinct words drawn
    at random.  The shared-cloud form of the batched workload."""
    g = rng_for(7, 0, 99)
    ns = log_uniform_int(g, lo, hi, nwords)
    kappa = g.uniform(1.5, 3.0, nwords)
    px = g.integers(0, nwords, npairs)
    py = (px + g.integers(1, nwords, npairs)) % nwords
    factor = lowrank_factor(d)

    def one(w):
        rng = rng_for(7, w, 0)
        return cloud_lowrank(rng, int(ns[w]), d, float(kappa[w]), random_unit(rng, d), factor).astype(np.float32)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        clouds = list(ex.map(one, range(nwords)))
    off = np.zeros(nwords, dtype=np.int64)
    off[1:] = np.cumsum(ns)[:-1]
    return Clouds(np.concatenate(clouds), off, ns.astype(np.int64), px.astype(np.int64), py.astype(np.int64),
                  np.full(npairs, B, dtype=np.int64),
                  meta=dict(workload="word_clouds", nwords=nwords, npairs=npairs, d=d))
