"""GPU: the benchmark's whole window (street 1216x352, N=6, K=32, 10 iterations) end to end
against the FP64 oracle's runs of the same window.

GEM is a stochastic search: per pixel, two runs part ways wherever the energy is flat to
the precision at hand (several candidates are then correct, and each pick changes the
predecessor slot of the rest of the chain), and the poses follow the depth.  How far two
equally valid runs land apart is measured on the oracle itself: the same window run with
three Philox keys (seed, seed + 1, seed + 2).  The oracle's runs take minutes on one host
core, so their results are stored by tests/golden/make_street_e2e.py (which calls only the
oracle and the input generator).  The GPU runs the window with the same three keys, and
what the window estimates is compared: log-likelihood, MIE energy, the median static
inverse-depth error against ground truth (raw and after median scaling), the pose error
against the true poses, the poses along the iterations, and the share of sampled pixels
whose inverse depth agrees with the oracle's run of the same key.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import gem as ogem
from paper_2104_06800_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "street_1216x352_n6_e2e.json")


def median_errors(rho, gt, static):
    ok = static & np.isfinite(rho) & (rho > 0) & np.isfinite(gt)
    raw = float(np.median(np.abs(rho[ok] - gt[ok]) / gt[ok]))
    s = np.median(gt[ok] / rho[ok])
    return raw, float(np.median(np.abs(rho[ok] * s - gt[ok]) / gt[ok]))


def summary(st, raw, scaled, pose_err):
    return np.array([st[0], st[1], raw, scaled, pose_err])


NAMES = ("loglik", "energy", "median error", "median error (scaled)", "pose error vs truth")


def test_street_window_end_to_end_against_oracle():
    from paper_2104_06800_amd.binding import Voldor
    gold = json.load(open(GOLDEN))
    runs = [gold] + gold["other_keys"]
    w = synth.make_window(2, 0)
    p0 = w["params"]
    lib = Voldor(0)
    gpu, ora = [], []
    for r in runs:
        p = dict(p0, seed=p0["seed"] + r["seed_offset"])
        b = lib.alloc(p, w["flow"], w["pose_init"])
        print(f"end to end: {p['W']}x{p['H']} N={p['N']} K={p['n_candidates']} key +{r['seed_offset']}", flush=True)
        lib.init_idepth(p, b)
        dposes = []
        for it in range(p["iters"]):
            lib.gem_step(p, b, it)
            torch.cuda.synchronize()
            dposes.append(float(np.abs(b["pose"].cpu().numpy() - np.array(r["pose_per_iter"][it])).max()))
        lib.finalize(p, b, p["iters"] - 1)
        torch.cuda.synchronize()
        rho = b["idepth"].cpu().numpy()
        st = b["stats"].cpu().numpy()
        raw, scaled = median_errors(rho, w["idepth_gt"], ~w["dynamic"])
        gpu.append(summary(st, raw, scaled, float(np.abs(b["pose"].cpu().numpy() - w["pose_gt"]).max())))
        ora.append(summary(r["stats"], r["median_static_rel_error"], r["median_static_rel_error_scaled"],
                           r["pose_err_vs_truth"]))
        print(f"  stats gpu {np.array2string(st[:6], precision=7)} oracle "
              f"{np.array2string(np.array(r['stats'][:6]), precision=7)}")
        if r["seed_offset"] == 0:
            # the statistics of the GPU's final state evaluated by the oracle: the final E-step,
            # the confidence and the sums (1e-4 as for the small windows)
            ob = ogem.alloc_buffers(p, w["flow"], b["pose"].cpu().numpy())
            ob["idepth"][...] = rho
            ost = ogem.finalize(p, ob, p["iters"] - 1)
            print(f"  oracle statistics of the GPU's final state: loglik {ost[0]:.9g} energy {ost[1]:.9g}")
            assert st[0] == pytest.approx(ost[0], rel=1e-4) and st[1] == pytest.approx(ost[1], rel=1e-4)
            assert abs(st[2] - ost[2]) <= 1e-4 * ost[2] and abs(st[5] - ost[5]) <= 1e-4 * ost[5]
        print("  pose difference from the oracle's run per iteration:", " ".join(f"{d:.1e}" for d in dposes))
        if "sample_index" in r:
            idx = np.array(r["sample_index"])
            srho = np.array(r["sample_idepth"])
            print(f"  sampled inverse depth within 1e-3 of the oracle's run: "
                  f"{np.mean(np.abs(rho.ravel()[idx] - srho) <= 1e-3 * srho):.4f}, within 1e-2: "
                  f"{np.mean(np.abs(rho.ravel()[idx] - srho) <= 1e-2 * srho):.4f}")
    lib.close()
    gpu, ora = np.array(gpu), np.array(ora)
    for i, n in enumerate(NAMES):
        print(f"{n:>24}: gpu {' '.join(f'{x:.6g}' for x in gpu[:, i])} | oracle {' '.join(f'{x:.6g}' for x in ora[:, i])}")
    # spread of equally valid runs: the oracle's keys about their mean
    om, gm = ora.mean(0), gpu.mean(0)
    spread = np.abs(ora - om).max(0)
    rel = np.abs(gm - om) / np.maximum(spread, 1e-12)
    print("mean gpu - mean oracle, in units of the oracle's largest deviation from its mean:",
          " ".join(f"{n} {x:.2f}" for n, x in zip(NAMES, rel)))
    # log-likelihood, depth errors and pose errors: within 3 times the spread of the oracle's
    # own runs; the MIE energy (weighted by each run's own final rigidness) within 3%
    keep = [0, 2, 3, 4]
    assert (rel[keep] <= 3.0).all(), rel
    assert np.abs(gpu[:, 1] / ora[:, 1] - 1).max() <= 3e-2
    assert np.abs(gpu[:, 0] / ora[:, 0] - 1).max() <= 2e-2
