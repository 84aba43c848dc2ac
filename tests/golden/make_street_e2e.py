"""Writes street_1216x352_n6_e2e.json: the FP64 oracle's plain GEM on the 1216x352, N=6
street window (input seed 2_000_000), 10 iterations from its Philox initial depth, then the
final E-step and statistics; and the same window run with two other Philox keys (seed + 1,
seed + 2), which are equally valid runs of the stochastic search and measure how far two
runs of it land apart.  Calls only the oracle and the input generator.

    python tests/golden/make_street_e2e.py

Stored per run: the statistics vector (log-likelihood, MIE energy, term counts, sum of C),
the poses after every iteration's pose step and their largest difference from the true
poses, the median static inverse-depth relative error against the generator's ground truth
(raw and after median scaling); for the first run also the final inverse depth and
confidence at 2048 seeded pixels.
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import gem  # noqa: E402
from paper_2104_06800_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "street_1216x352_n6_e2e.json")


def median_errors(rho, gt, static):
    ok = static & np.isfinite(rho) & (rho > 0) & np.isfinite(gt)
    raw = float(np.median(np.abs(rho[ok] - gt[ok]) / gt[ok]))
    s = np.median(gt[ok] / rho[ok])
    return raw, float(np.median(np.abs(rho[ok] * s - gt[ok]) / gt[ok]))


def run(seed_offset):
    w = synth.make_window(2, 0)
    p = dict(w["params"])
    p["seed"] = p["seed"] + seed_offset
    b = gem.alloc_buffers(p, w["flow"], w["pose_init"])
    gem.init_idepth(p, b)
    poses = []
    t0 = time.time()
    for it in range(p["iters"]):
        gem.gem_step(p, b, it)
        poses.append(b["pose"].tolist())
        print(f"key +{seed_offset}: iteration {it} done, {time.time() - t0:.0f} s", flush=True)
    st = gem.finalize(p, b, p["iters"] - 1)
    raw, scaled = median_errors(b["idepth"], w["idepth_gt"], ~w["dynamic"])
    out = dict(seed_offset=seed_offset, stats=[float(x) for x in st], pose_per_iter=poses,
               pose_err_vs_truth=float(np.abs(b["pose"] - w["pose_gt"]).max()),
               median_static_rel_error=raw, median_static_rel_error_scaled=scaled)
    if seed_offset == 0:
        H, W = p["H"], p["W"]
        idx = np.sort(np.random.default_rng(0).choice(H * W, 2048, replace=False))
        out.update(sample_index=idx.tolist(), sample_idepth=[float(x) for x in b["idepth"].ravel()[idx]],
                   sample_conf=[float(x) for x in b["conf"].ravel()[idx]])
    return out


def main():
    with ProcessPoolExecutor(3) as ex:
        runs = list(ex.map(run, [0, 1, 2]))
    out = dict(workload="street 1216x352, N=6, K=32, 10 iterations, input seed 2000000",
               iters=len(runs[0]["pose_per_iter"]), **runs[0], other_keys=runs[1:])
    with open(OUT, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    for r in runs:
        print(f"key +{r['seed_offset']}: loglik {r['stats'][0]:.9g} energy {r['stats'][1]:.9g} error "
              f"{r['median_static_rel_error']:.4f} / {r['median_static_rel_error_scaled']:.4f} pose vs truth "
              f"{r['pose_err_vs_truth']:.2e}")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
