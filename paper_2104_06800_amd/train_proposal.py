"""Trains the learned proposal on plain-GEM targets of seeded synthetic windows and compares
learned-initialised GEM with plain GEM on held-out windows.

  python -m paper_2104_06800_amd.train_proposal --train 256 --test 8 --steps 2000 \\
      --out proposal_n6.npz

Windows: the 640x480, N = 6 street recipe; training seeds k = 0..train-1, held-out seeds
k = 10^6 .. 10^6 + test - 1.  The weights file holds the FP32 parameters and the run's
settings, loss history and held-out comparison.
"""
import argparse
import json
import time

import numpy as np


def log(*a):
    print(*a, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=256)
    ap.add_argument("--test", type=int, default=8)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--lam", type=float, default=0.1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", required=True)
    ap.add_argument("--weights", default=None, help="evaluate these weights instead of training")
    args = ap.parse_args()

    from . import proposal as pr

    t0 = time.time()
    import torch
    from .binding import Voldor
    test_w = pr.generate(list(range(pr.TEST_SEED0, pr.TEST_SEED0 + args.test)), args.workers)
    log(f"generated {len(test_w)} held-out windows ({time.time() - t0:.0f} s)")
    meta = {}
    if args.weights:
        params, meta = pr.load(args.weights)
        meta = {k: v for k, v in meta.items() if k not in ("compare", "summary", "compare_cold", "summary_cold")}
        lib = Voldor(0)
    else:
        train_w = []
        ks = list(range(pr.TRAIN_SEED0, pr.TRAIN_SEED0 + args.train))
        for i in range(0, len(ks), 32):
            train_w += pr.generate(ks[i:i + 32], args.workers)
            log(f"generated {len(train_w)}/{len(ks)} training windows ({time.time() - t0:.0f} s)")
        lib = Voldor(0)
        data = pr.Dataset(lib, train_w)
        del train_w
        errs = [it["err_gem"] for it in data.items]
        log(f"plain-GEM targets ready ({time.time() - t0:.0f} s); plain GEM error on training windows: "
            f"median {np.median(errs):.4f}")
        params, hist = pr.train(lib, data, args.steps, lr=args.lr, lr_final=args.lr_final, lam=args.lam,
                                seed=args.seed)
        log(f"trained ({time.time() - t0:.0f} s)")
        meta = dict(train=args.train, steps=args.steps, lr=args.lr, lr_final=args.lr_final, lam=args.lam,
                    seed=args.seed, loss_history=hist)
    net = lib.net_alloc(params)
    for warm in (True, False):
        res = pr.compare(lib, net, test_w, warm=warm)
        summ = pr.summarize(res)
        tag = "warm" if warm else "cold"
        for i, r in enumerate(res):
            log(f"[{tag}] held-out {i}: plain {r['err_plain']:.4f} ({r['ms_plain']:.2f} ms); proposal "
                f"{r['err_proposal']:.4f} ({r['ms_proposal']:.2f} ms); learned start after k iterations: "
                f"{' '.join(f'{e:.4f}' for e in r['err_learned'])}")
        log(f"[{tag}] summary: {json.dumps(summ)}")
        meta["compare" if warm else "compare_cold"] = json.dumps(res)
        meta["summary" if warm else "summary_cold"] = json.dumps(summ)
    meta["test"] = args.test
    pr.save(args.out, params, meta)
    log(f"saved {args.out}")
    lib.close()


if __name__ == "__main__":
    main()
