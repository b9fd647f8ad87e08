"""The learned permutation-budget allocator at the size of its workload.

Usage: ``python -m paper_2605_08048_amd.budget_run [--train 20000] [--test 4096]``
(one GPU; prints one JSON summary).

The network (12 -> 64 -> 64 -> 2) is trained on the null-statistic spreads
the method itself produces: every training pair is tested with the full
budget (20,000 splits) and its (mean, log sd) of T_b is the target.  On
held-out pairs it is compared with

* the fixed budget of the paper (every pair at b_max splits; done twice with
  independent seeds, whose decisions at alpha differ only by Monte Carlo
  noise), and
* the same three-stage procedure without the network (every pair at b_min
  splits, the exact fallback band rerun at b_max).

The adaptive runs use a seed independent of both reference runs.  Pairs
come from the learned-budget workload generator (d = 768, n and m
log-uniform on [20, 2000], half of the pairs null), generated and processed
in chunks so that host memory stays bounded.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _chunks(a, b, k):
    for s in range(a, b, k):
        yield range(s, min(s + k, b))


def run(train=20000, test=4096, d=768, b_train=20000, b_max=20000, alpha=0.05, chunk=2048, steps=1500,
        lr=3e-3, b_min=200, net_b_min=16, net_b_first=1, p_lo=0.02, p_hi=0.10, log=print):
    import torch

    from . import allocator as A
    from . import hbt, synth

    dev = torch.device("cuda:0")
    total = train + test
    t0 = time.perf_counter()
    feats, targs = [], []
    gpu_train = 0.0
    for rg in _chunks(0, train, chunk):
        b = synth.budget_batch_4096(npairs=total, d=d, B=b_train, limit=rg)
        Z = torch.from_numpy(b.Z).to(dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = hbt.perm_test_batched(Z, b.row_offset, b.n, b.m, b.B, seed=11,
                                    pair_index=np.arange(rg.start, rg.stop, dtype=np.uint32), sync=False)
        feats.append(hbt.budget_features(res, d))
        targs.append(hbt.null_targets(res))
        torch.cuda.synchronize()
        gpu_train += time.perf_counter() - t
        del Z
        log(f"training targets: pairs {rg.start}..{rg.stop - 1} done ({time.perf_counter() - t0:.0f} s)")
    F, T = torch.cat(feats), torch.cat(targs)
    al = A.Allocator.create(dev, seed=0)
    t = time.perf_counter()
    losses = al.fit(F, T, steps=steps, lr=lr)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t
    log(f"trained: loss {losses[0]:.4g} -> {losses[-1]:.4g} in {fit_s:.1f} s")
    tot = dict(fixed=0, net=0, base=0, dis_full=0, dis_net=0, dis_base=0, rejections=0, pairs=0,
               net_stage3=0, base_stage3=0, sec_fixed=0.0, sec_net=0.0, sec_base=0.0)
    mse_net, mse_const = np.zeros(2), np.zeros(2)
    const = T.cpu().numpy().astype(np.float64).mean(0)
    for rg in _chunks(train, total, chunk):
        b = synth.budget_batch_4096(npairs=total, d=d, B=b_max, limit=rg)
        Z = torch.from_numpy(b.Z).to(dev)
        P = b.npairs
        off, nn, mm = b.row_offset, b.n, b.m

        def timed(f):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = f()
            torch.cuda.synchronize()
            return r, time.perf_counter() - t

        full_a, sa = timed(lambda: hbt.perm_test_batched(Z, off, nn, mm, np.full(P, b_max), seed=21))
        full_b, _ = timed(lambda: hbt.perm_test_batched(Z, off, nn, mm, np.full(P, b_max), seed=22))
        net, sn = timed(lambda: A.adaptive_perm_test(Z, off, nn, mm, al, d=d, seed=31, b_min=net_b_min,
                                                     b_first=net_b_first, b_max=b_max, p_lo=p_lo, p_hi=p_hi))
        base, sb = timed(lambda: A.adaptive_perm_test(Z, off, nn, mm, None, d=d, seed=31, b_min=b_min,
                                                      b_max=b_max, p_lo=p_lo, p_hi=p_hi))
        # the network's estimate of the null (mean, log sd) against the truth
        res1 = hbt.perm_test_batched(Z, off, nn, mm, np.full(P, 1), seed=31, sync=False)
        pred = al.predict(hbt.budget_features(res1, d)).cpu().numpy().astype(np.float64)
        truth = np.stack([full_a["t_mean"], np.log(full_a["t_sd"])], 1)
        mse_net += np.sum((pred - truth) ** 2, 0)
        mse_const += np.sum((const - truth) ** 2, 0)
        Da, Db = full_a["p"] < alpha, full_b["p"] < alpha
        tot["fixed"] += P * b_max
        tot["net"] += net["splits"]["total"]
        tot["base"] += base["splits"]["total"]
        tot["net_stage3"] += net["splits"]["stage3"]
        tot["net_pairs_at_b_max_stage2"] = tot.get("net_pairs_at_b_max_stage2", 0) + \
            net["splits"]["pairs_at_b_max_before_stage3"]
        tot["pairs_truly_in_band"] = tot.get("pairs_truly_in_band", 0) + \
            int(np.sum((full_a["p"] >= p_lo) & (full_a["p"] <= p_hi)))
        tot["base_stage3"] += base["splits"]["stage3"]
        tot["dis_full"] += int(np.sum(Da != Db))
        tot["dis_net"] += int(np.sum((net["p"] < alpha) != Da))
        tot["dis_base"] += int(np.sum((base["p"] < alpha) != Da))
        tot["rejections"] += int(Da.sum())
        tot["pairs"] += P
        tot["sec_fixed"] += sa
        tot["sec_net"] += sn
        tot["sec_base"] += sb
        del Z
        log(f"held-out pairs {rg.start}..{rg.stop - 1} done ({time.perf_counter() - t0:.0f} s)")
    tot["mse_net"] = (mse_net / tot["pairs"]).tolist()
    tot["mse_constant"] = (mse_const / tot["pairs"]).tolist()
    tot.update(train_pairs=train, test_pairs=test, d=d, b_train=b_train, b_max=b_max, alpha=alpha,
               b_min=b_min, net_b_min=net_b_min, net_b_first=net_b_first, band=[p_lo, p_hi],
               loss_first=losses[0], loss_last=losses[-1], fit_steps=steps, fit_s=fit_s,
               gpu_s_training_targets=gpu_train, wall_s=time.perf_counter() - t0)
    return tot


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--test", type=int, default=4096)
    ap.add_argument("--d", type=int, default=768)
    ap.add_argument("--b-train", type=int, default=20000)
    ap.add_argument("--b-max", type=int, default=20000)
    ap.add_argument("--chunk", type=int, default=2048)
    ap.add_argument("--steps", type=int, default=1500)
    a = ap.parse_args()
    out = run(train=a.train, test=a.test, d=a.d, b_train=a.b_train, b_max=a.b_max, chunk=a.chunk, steps=a.steps,
              log=lambda s: print(f"[budget] {s}", file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
